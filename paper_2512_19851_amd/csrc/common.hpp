// Shared host/device helpers of libsten: status handling, argument checks and
// the XCD-aware tile map. Internal header (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sten.h"

namespace sten {

// Wave size of CDNA (gfx9 family): 64 lanes.
constexpr int kWave = 64;
// MI355X has 8 accelerator complex dies (XCDs); consecutive workgroups of a
// launch are dealt round-robin across them.
constexpr uint32_t kNumXcd = 8;

// Record a failed HIP call for sten_last_hip_error() and map it to a status.
sten_status hip_fail(hipError_t e);

// Check the sticky launch error after enqueuing kernels.
sten_status check_launch();

// True if p is device memory (or managed memory) usable on the current device.
// Clears the HIP error state if the query itself fails.
bool is_device_ptr(const void* p);

// Bytes spanned by an H x W grid with row stride ld (0 when empty).
inline size_t span_bytes(int64_t H, int64_t W, int64_t ld, size_t esize) {
    if (H <= 0 || W <= 0) return 0;
    return (size_t)((H - 1) * ld + W) * esize;
}

// True if [a, a+na) and [b, b+nb) intersect (empty ranges never do).
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (na == 0 || nb == 0 || a == nullptr || b == nullptr) return false;
    uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

// Common checks of the plain-grid calls: sizes, strides, pointers, aliasing.
// `need_work` says whether the work buffer takes part in this call.
sten_status check_grid_args(const void* u0, const void* out, const void* work, bool need_work,
                            int64_t H, int64_t W, int64_t ld, int32_t T, size_t esize);

// Workgroup b of nb -> tile index, giving XCD x = b mod 8 the contiguous tile
// range [x*per + min(x, extra), ...). Bijective on [0, nb).
__host__ __device__ inline uint32_t xcd_tile_of_block(uint32_t b, uint32_t nb) {
    uint32_t xcd = b % kNumXcd;
    uint32_t local = b / kNumXcd;
    uint32_t per = nb / kNumXcd;
    uint32_t extra = nb % kNumXcd;
    return xcd * per + (xcd < extra ? xcd : extra) + local;
}

inline uint32_t ceil_div(int64_t a, int64_t b) { return (uint32_t)((a + b - 1) / b); }

// One grid of a multi-grid launch: an H x W grid with row stride ld, read from
// `in`, written to `out` (interior only).
template <typename T>
struct GridView {
    const T* in;
    T* out;
    int H, W;
    int64_t ld;
};

// Most sweeps per launch of the streaming blocked kernel: FP64 launches of 13
// and 14 sweeps run at 2 waves per SIMD (their rows do not fit the registers
// of 3); FP32 stops at 12.
constexpr int kMaxStreamLevelsF64 = 14;
constexpr int kMaxStreamLevelsF32 = 12;
template <typename T>
constexpr int max_stream_levels() { return sizeof(T) == 8 ? kMaxStreamLevelsF64 : kMaxStreamLevelsF32; }

// Streaming blocked kernel on several FP64 grids at once (temporal.hip), up to
// kMaxStreamGridsPerLaunch grids per launch.
constexpr int kMaxStreamGridsPerLaunch = 32;
// Returns false, with nothing launched, for levels outside 1..12.
bool launch_stream_grids_f64(const GridView<double>* views, int n, double c, int levels, hipStream_t s);

// One sweep of each of n FP64 grids (sweep.hip), in launches of up to 32
// grids. Every grid: H, W >= 3, 16-byte aligned, even ld; returns false, with
// nothing launched, otherwise.
// Ghost cells of the four neighbours' output views that mirror a grid's first
// and last interior rows and columns, so that one sweep also does the ghost
// exchange of depth 1 (NULL where there is no neighbour). Neighbours share
// column (north, south) or row (west, east) coordinates with the grid.
struct GridMirror {
    double* north = nullptr;  // the north neighbour's last view row
    double* south = nullptr;  // the south neighbour's first view row
    double* west = nullptr;   // the west neighbour's last view column (row stride ld_west)
    double* east = nullptr;   // the east neighbour's first view column (row stride ld_east)
    int64_t ld_west = 0, ld_east = 0;
};
// With mirrors (one per view), each sweep also stores grid k's edge rows and
// columns into mirrors[k]'s ghost cells.
bool launch_sweep_grids_f64(const GridView<double>* views, int n, double c, hipStream_t s,
                            const GridMirror* mirrors = nullptr);

}  // namespace sten
