// Pieces shared by the streaming blocked kernels (the five-point Jacobi
// method and the cavity flow's pressure iteration): vector types, DPP lane
// shifts, clamped row loads and branch-free row stores. Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sten {
namespace stream {

template <typename T, int V>
struct TVec;
template <>
struct TVec<double, 2> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct TVec<float, 4> {
    typedef float type __attribute__((ext_vector_type(4)));
};

// BEGIN KERNEL SOURCE (the HBM traffic measurement is keyed to this region)
// Lane l receives lane l-1's value; lane 0 receives 0 (DPP wave shift right by
// 1, bound control set, so no register has to be cleared first).
__device__ __forceinline__ int lane_from_lower_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }
// Lane l receives lane l+1's value; lane 63 receives 0 (DPP wave shift left by 1).
__device__ __forceinline__ int lane_from_upper_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }

__device__ __forceinline__ float lane_from_lower(float v) {
    return __builtin_bit_cast(float, lane_from_lower_i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float lane_from_upper(float v) {
    return __builtin_bit_cast(float, lane_from_upper_i(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_from_lower(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)lane_from_lower_i((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)lane_from_lower_i((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double lane_from_upper(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)lane_from_upper_i((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)lane_from_upper_i((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Strip kinds: EDGE 0, a strip whose loaded columns are all interior (no
// column test at all); EDGE 1, a strip that touches the grid's first or last
// column but loads only columns inside the grid; EDGE 2, a strip whose loads
// may leave the grid (columns clamped, stored column by column).

// Row r (clamped into the grid) of the input into x: V consecutive columns
// from j0. EDGE 2 strips load column by column with the column clamped into
// the grid as well: a column outside the grid never reaches an interior point
// (an interior column reads only its two neighbours, both inside the grid), so
// its value is irrelevant and no lane needs a branch.
template <typename T, int V, int EDGE>
__device__ __forceinline__ void stream_load(const T* __restrict__ in, int r, int H, int W, int64_t ld, int j0,
                                            T (&x)[V]) {
    typedef typename TVec<T, V>::type VT;
    r = min(max(r, 0), H - 1);
    const T* row = in + (int64_t)r * ld;
    if constexpr (EDGE < 2) {
        const VT v = *reinterpret_cast<const VT*>(row + j0);
#pragma unroll
        for (int e = 0; e < V; ++e) x[e] = v[e];
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) x[e] = row[min(max(j0 + e, 0), W - 1)];
    }
}

// Store one finished row (level TL) through a buffer resource that spans
// just that row: lanes that store nothing get an offset past the row's end,
// which the hardware drops, and a step past the band (live == false) gets an
// empty range. No lane branches, so the compiler can count every store in
// flight and never waits for a younger load than the one a step reads.
// EDGE 0 and 1 strips store whole vectors; EDGE 2 strips store column by column.
constexpr uint32_t kDropOffset = 0x80000000u;  // past the end of any row range
constexpr int kRawBufferConfig = 0x00020000;    // raw (untyped) buffer words, gfx9 family

template <typename T, int V, int EDGE>
__device__ __forceinline__ void stream_store(T* __restrict__ out, int r, int64_t ld, int W, bool live,
                                             uint32_t voff_vec, const uint32_t (&voff_el)[V], const T (&top)[V]) {
    T* row = out + (int64_t)(live ? r : 1) * ld;  // a dead step's row may lie outside the grid
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(row, 0, live ? W * (int)sizeof(T) : 0, kRawBufferConfig);
    if constexpr (EDGE < 2) {
        typedef int IV __attribute__((ext_vector_type(4)));
        static_assert(sizeof(T) * V == sizeof(IV), "one 16-byte vector per lane");
        typedef typename TVec<T, V>::type VT;
        VT v;
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = top[e];
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(IV, v), rs, (int)voff_vec, 0, 0);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if constexpr (sizeof(T) == 8) {
                typedef int IV2 __attribute__((ext_vector_type(2)));
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(IV2, top[e]), rs, (int)voff_el[e], 0, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, top[e]), rs, (int)voff_el[e], 0, 0);
            }
        }
    }
}

// END KERNEL SOURCE

}  // namespace stream
}  // namespace sten
