// Temporal blocking of the five-point Jacobi method: TL sweeps per pass over
// HBM, bit-identical to TL single sweeps.
//
// A workgroup is one wave. It owns an output tile of ROWS rows by
// 64*V - 2*HALO columns (HALO = TL rounded up to a multiple of V, so every
// vector stays aligned) and loads the tile grown by TL rows and HALO columns
// on every side (lane l holds V consecutive columns of each loaded row). It then
// applies TL sweeps in registers: after sweep s the values are exact on the
// loaded block shrunk by s on every side, because every point needs only its
// four neighbours from sweep s-1. The central block, exact after TL sweeps,
// is stored. Points on the grid's boundary ring keep their value at every
// level; points outside the grid are loaded as 0 and only ever feed values
// that are not stored.
//
// Each point of each level is computed exactly as in the single-sweep kernel,
// c * (((N + S) + W) + E), so the result is bit-identical; HBM traffic per
// sweep drops from 16 B (FP64) to about 16/TL B per interior point, at the cost
// of recomputing the halo (rows: 2*TL per ROWS, columns: 2*TL per 64*V) and
// re-reading halo rows from L2.
#include <algorithm>

#include "common.hpp"

namespace sten {
namespace {

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
template <typename T, int V, int ROWS, int TL>
__global__ __launch_bounds__(64) void sweep_tb_kernel(const T* __restrict__ in, T* __restrict__ out, int H, int W,
                                                     int64_t ld, T c, uint32_t strips) {
    constexpr int NR = ROWS + 2 * TL;                 // loaded rows
    constexpr int HALO = (TL + V - 1) / V * V;        // halo columns, a multiple of V (aligned vectors)
    constexpr int OW = 64 * V - 2 * HALO;             // output columns per tile
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t band = tile / strips;
    const uint32_t strip = tile - band * strips;
    const int lane = threadIdx.x;
    const int cs = (int)strip * OW - HALO;  // first loaded column (may be negative), a multiple of V
    const int j0 = cs + lane * V;         // this lane's first column
    const int rb = 1 + (int)band * ROWS;  // first output row
    const int r0 = rb - TL;               // first loaded row (may be negative)

    typedef typename TVec<T, V>::type VT;
    T a[NR][V];
    const bool lane_full = (j0 >= 0) && (j0 + V <= W);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = r0 + k;
        if (r >= 0 && r < H) {
            const T* row = in + (int64_t)r * ld;
            if (lane_full) {
                const VT x = *reinterpret_cast<const VT*>(row + j0);
#pragma unroll
                for (int e = 0; e < V; ++e) a[k][e] = x[e];
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) a[k][e] = (j0 + e >= 0 && j0 + e < W) ? row[j0 + e] : T(0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) a[k][e] = T(0);
        }
    }
    bool col_in[V];
#pragma unroll
    for (int e = 0; e < V; ++e) col_in[e] = (j0 + e >= 1) && (j0 + e <= W - 2);

#pragma unroll
    for (int s = 1; s <= TL; ++s) {
        // rows s-1 .. NR-s are still exact; update rows s .. NR-1-s in place, top to bottom
        T prev[V];
#pragma unroll
        for (int e = 0; e < V; ++e) prev[e] = a[s - 1][e];
#pragma unroll
        for (int k = s; k <= NR - 1 - s; ++k) {
            const int r = r0 + k;
            const bool row_in = (r >= 1) && (r <= H - 2);
            const T lft = __shfl_up(a[k][V - 1], 1);   // column j0 - 1
            const T rgt = __shfl_down(a[k][0], 1);     // column j0 + V
            T nv[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const T west = (e == 0) ? lft : a[k][e > 0 ? e - 1 : 0];
                const T east = (e == V - 1) ? rgt : a[k][e < V - 1 ? e + 1 : 0];
                T sum = prev[e] + a[k + 1][e];  // N + S
                sum = sum + west;               // + W
                sum = sum + east;               // + E
                nv[e] = (row_in && col_in[e]) ? c * sum : a[k][e];
            }
#pragma unroll
            for (int e = 0; e < V; ++e) {
                prev[e] = a[k][e];
                a[k][e] = nv[e];
            }
        }
    }

    // store rows TL .. TL+ROWS-1 of the tile, columns [cs + HALO, cs + HALO + OW), interior only
    const int oc0 = cs + HALO;
#pragma unroll
    for (int k = TL; k < TL + ROWS; ++k) {
        const int r = r0 + k;
        if (r >= 1 && r <= H - 2) {
            T* row = out + (int64_t)r * ld;
            const bool inner = (j0 >= oc0) && (j0 + V <= oc0 + OW) && (j0 >= 1) && (j0 + V <= W - 1);
            if (inner) {
                VT x;
#pragma unroll
                for (int e = 0; e < V; ++e) x[e] = a[k][e];
                *reinterpret_cast<VT*>(row + j0) = x;
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int j = j0 + e;
                    if (j >= oc0 && j < oc0 + OW && j >= 1 && j <= W - 2) row[j] = a[k][e];
                }
            }
        }
    }
}

// END KERNEL SOURCE

template <typename T>
__global__ void tb_ring_copy_kernel(const T* __restrict__ u0, T* __restrict__ d1, T* __restrict__ d2, int H, int W,
                                    int64_t ld) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nring = 2 * (int64_t)W + 2 * (int64_t)(H - 2);
    if (idx >= nring) return;
    int i, j;
    if (idx < W) {
        i = 0;
        j = (int)idx;
    } else if (idx < 2 * (int64_t)W) {
        i = H - 1;
        j = (int)(idx - W);
    } else {
        const int64_t r = idx - 2 * (int64_t)W;
        i = 1 + (int)(r >> 1);
        j = (r & 1) ? W - 1 : 0;
    }
    const int64_t off = (int64_t)i * ld + j;
    d1[off] = u0[off];
    if (d2 != nullptr) d2[off] = u0[off];
}

template <typename T, int V, int ROWS, int TL>
void launch_tb(const T* in, T* out, int H, int W, int64_t ld, T c, hipStream_t s) {
    constexpr int HALO = (TL + V - 1) / V * V;
    constexpr int OW = 64 * V - 2 * HALO;
    const uint32_t strips = ceil_div(W, OW);
    const uint32_t bands = ceil_div(H - 2, ROWS);
    sweep_tb_kernel<T, V, ROWS, TL><<<strips * bands, 64, 0, s>>>(in, out, H, W, ld, c, strips);
}

int g_tb_rows = 0;  // tuning hook: output rows per tile (0: 8)

template <typename T, int V, int ROWS>
void launch_levels_rows(const T* in, T* out, int H, int W, int64_t ld, T c, int levels, hipStream_t s) {
    switch (levels) {
        case 1: launch_tb<T, V, ROWS, 1>(in, out, H, W, ld, c, s); break;
        case 2: launch_tb<T, V, ROWS, 2>(in, out, H, W, ld, c, s); break;
        case 3: launch_tb<T, V, ROWS, 3>(in, out, H, W, ld, c, s); break;
        case 4: launch_tb<T, V, ROWS, 4>(in, out, H, W, ld, c, s); break;
        case 5: launch_tb<T, V, ROWS, 5>(in, out, H, W, ld, c, s); break;
        default: launch_tb<T, V, ROWS, 6>(in, out, H, W, ld, c, s); break;
    }
}

// One blocked launch of `levels` sweeps (1..6).
template <typename T, int V>
void launch_levels(const T* in, T* out, int H, int W, int64_t ld, T c, int levels, hipStream_t s) {
    switch (g_tb_rows) {
        case 4: launch_levels_rows<T, V, 4>(in, out, H, W, ld, c, levels, s); break;
        case 12: launch_levels_rows<T, V, 12>(in, out, H, W, ld, c, levels, s); break;
        case 16: launch_levels_rows<T, V, 16>(in, out, H, W, ld, c, levels, s); break;
        default: launch_levels_rows<T, V, 8>(in, out, H, W, ld, c, levels, s); break;
    }
}

template <typename T>
sten_status run_tb(const T* u0, T* out, T* work, int64_t H, int64_t W, int64_t ld, int32_t T_, T c, int32_t tl,
                   hipStream_t stream) {
    if (tl < 1 || tl > 6) return STEN_ERR_ARG;
    const bool interior = H >= 3 && W >= 3;
    const int launches = (T_ + tl - 1) / tl;
    const bool need_work = interior && launches >= 2;
    sten_status st = check_grid_args(u0, out, work, need_work, H, W, ld, T_, sizeof(T));
    if (st != STEN_OK || H == 0 || W == 0) return st;
    constexpr int VV = 16 / (int)sizeof(T);
    if (!interior || T_ == 0 || (((uintptr_t)u0 | (uintptr_t)out | (need_work ? (uintptr_t)work : 0)) % 16) != 0 ||
        ld % VV != 0)
        return STEN_ERR_UNSUPPORTED;  // the caller uses the single-sweep path for these
    const int h = (int)H, w = (int)W;
    const int64_t nring = 2 * W + 2 * (H - 2);
    tb_ring_copy_kernel<T><<<ceil_div(nring, 256), 256, 0, stream>>>(u0, out, need_work ? work : nullptr, h, w, ld);
    // launch k (1-based) applies `lev` sweeps; the last launch must write `out`
    const T* src = u0;
    int done = 0;
    for (int k = 1; k <= launches; ++k) {
        const int lev = std::min(tl, T_ - done);
        T* dst = ((launches - k) % 2 == 0) ? out : work;
        launch_levels<T, VV>(src, dst, h, w, ld, c, lev, stream);
        done += lev;
        src = dst;
    }
    return check_launch();
}

}  // namespace

// Entry used by the plain calls when they pick the blocked schedule.
sten_status run_tb_f64(const double* u0, double* out, double* work, int64_t H, int64_t W, int64_t ld, int32_t T,
                       double c, int32_t levels, hipStream_t stream) {
    return run_tb<double>(u0, out, work, H, W, ld, T, c, levels, stream);
}
sten_status run_tb_f32(const float* u0, float* out, float* work, int64_t H, int64_t W, int64_t ld, int32_t T,
                       float c, int32_t levels, hipStream_t stream) {
    return run_tb<float>(u0, out, work, H, W, ld, T, c, levels, stream);
}

}  // namespace sten

extern "C" {

sten_status sten_jacobi5_f64_tb(const double* u0, double* out, double* work, int64_t H, int64_t W, int64_t ld,
                                int32_t T, double c, int32_t levels, hipStream_t stream) {
    return sten::run_tb<double>(u0, out, work, H, W, ld, T, c, levels, stream);
}

sten_status sten_jacobi5_f32_tb(const float* u0, float* out, float* work, int64_t H, int64_t W, int64_t ld,
                                int32_t T, float c, int32_t levels, hipStream_t stream) {
    return sten::run_tb<float>(u0, out, work, H, W, ld, T, c, levels, stream);
}

sten_status sten_tune_tb_rows(int32_t rows) {
    if (rows != 0 && rows != 4 && rows != 8 && rows != 12 && rows != 16) return STEN_ERR_ARG;
    sten::g_tb_rows = rows;
    return STEN_OK;
}

}  // extern "C"
