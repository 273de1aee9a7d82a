// Plain five-point Jacobi sweep (listing of the 2-D Laplace solver,
// Section III-A): out[i,j] = c * (((in[i-1,j] + in[i+1,j]) + in[i,j-1]) + in[i,j+1])
// on the interior, iterated T times with a ping-pong swap.
//
// Kernel design (gfx950, HBM-bound: 4 flop per 16 B in FP64):
//  * A workgroup of 256 lanes (4 waves) owns a tile of ROWS output rows by
//    256*V columns. Each lane owns V consecutive columns (one 16-byte vector:
//    2 doubles or 4 floats), so every row load of a wave is a coalesced 1 KiB
//    global_load_dwordx4.
//  * The lane loads its column vector for all ROWS+2 input rows up front
//    (ROWS+2 independent 16-byte loads in flight per lane), then walks down:
//    up/down neighbours come from the lane's own registers, left/right
//    neighbours of the vector's end elements from the adjacent lanes through a
//    cross-lane shuffle; only the wave's two edge lanes issue one extra scalar
//    load per row. Each input element is read from HBM once per tile; the two
//    halo rows are shared with the vertically adjacent tiles through L2.
//  * Tiles are mapped to workgroups so that each XCD walks a contiguous band
//    of rows, keeping halo rows in that XCD's L2.
//  * The arithmetic is exactly the listing's order with one rounding per
//    operation; the library is built with -ffp-contract=off.
#include <algorithm>
#include <atomic>

#include "common.hpp"

namespace sten {

bool launch_levels_f64(const double* in, double* out, int H, int W, int64_t ld, double c, int levels,
                       hipStream_t s);
sten_status run_tb_f64(const double* u0, double* out, double* work, int64_t H, int64_t W, int64_t ld, int32_t T,
                       double c, int32_t levels, hipStream_t stream);
sten_status run_tb_f32(const float* u0, float* out, float* work, int64_t H, int64_t W, int64_t ld, int32_t T,
                       float c, int32_t levels, hipStream_t stream);

namespace {

// BEGIN KERNEL SOURCE (the HBM traffic measurement is keyed to this region)
constexpr int kBlock = 256;

template <typename T, int V>
struct Vec;
template <typename T>
struct Vec<T, 1> {
    typedef T type;
};
template <>
struct Vec<double, 2> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec<float, 4> {
    typedef float type __attribute__((ext_vector_type(4)));
};

// Load columns [jb, jb+V) of one row; columns at or beyond W read as 0.
template <typename T, int V>
__device__ __forceinline__ void load_vec(const T* __restrict__ row, int jb, int W, T (&v)[V]) {
    if constexpr (V == 1) {
        v[0] = (jb < W) ? row[jb] : T(0);
    } else {
        if (jb + V <= W) {
            typedef typename Vec<T, V>::type VT;
            VT x = *reinterpret_cast<const VT*>(row + jb);
#pragma unroll
            for (int e = 0; e < V; ++e) v[e] = x[e];
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) v[e] = (jb + e < W) ? row[jb + e] : T(0);
        }
    }
}

// Store columns [jb, jb+V) of one row, skipping the ring columns 0 and W-1
// and anything at or beyond W.
template <typename T, int V>
__device__ __forceinline__ void store_vec(T* __restrict__ row, int jb, int W, const T (&v)[V]) {
    if constexpr (V > 1) {
        if (jb >= 1 && jb + V <= W - 1) {
            typedef typename Vec<T, V>::type VT;
            VT x;
#pragma unroll
            for (int e = 0; e < V; ++e) x[e] = v[e];
            *reinterpret_cast<VT*>(row + jb) = x;
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
        int j = jb + e;
        if (j >= 1 && j <= W - 2) row[j] = v[e];
    }
}

// One tile of the sweep. FULL: the tile has ROWS output rows and every lane of
// the wave lies inside the grid (jb + V <= W), so loads need no guards.
template <typename T, int V, int ROWS, bool FULL>
__device__ __forceinline__ void sweep_tile(const T* __restrict__ src, T* __restrict__ dst, int n, int jb,
                                           int lane, int W, int64_t ld, T c) {
    T r[ROWS + 2][V];
#pragma unroll
    for (int k = 0; k < ROWS + 2; ++k) {
        if (FULL) {
            typedef typename Vec<T, V>::type VT;
            if constexpr (V == 1) {
                r[k][0] = src[(int64_t)k * ld + jb];
            } else {
                VT x = *reinterpret_cast<const VT*>(src + (int64_t)k * ld + jb);
#pragma unroll
                for (int e = 0; e < V; ++e) r[k][e] = x[e];
            }
        } else if (k < n + 2) {
            load_vec<T, V>(src + (int64_t)k * ld, jb, W, r[k]);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) r[k][e] = T(0);
        }
    }
    // The wave's edge lanes fetch the one neighbour that lies in another wave.
    T el[ROWS], er[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        el[k] = T(0);
        er[k] = T(0);
        if (FULL || k < n) {
            const T* row = src + (int64_t)(k + 1) * ld;
            if (lane == 0 && jb > 0 && jb <= W) el[k] = row[jb - 1];
            if (lane == kWave - 1 && jb + V < W) er[k] = row[jb + V];
        }
    }
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        if (FULL || k < n) {  // n is uniform over the block, so whole waves shuffle together
            T left0 = __shfl_up(r[k + 1][V - 1], 1);
            T rightv = __shfl_down(r[k + 1][0], 1);
            if (lane == 0) left0 = el[k];
            if (lane == kWave - 1) rightv = er[k];
            T o[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const T west = (e == 0) ? left0 : r[k + 1][e > 0 ? e - 1 : 0];
                const T east = (e == V - 1) ? rightv : r[k + 1][e < V - 1 ? e + 1 : 0];
                T s = r[k][e] + r[k + 2][e];  // N + S
                s = s + west;                 // + W
                s = s + east;                 // + E
                o[e] = c * s;
            }
            store_vec<T, V>(dst + (int64_t)k * ld, jb, W, o);
        }
    }
}

template <typename T, int V, int ROWS>
__global__ __launch_bounds__(kBlock) void sweep_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                       int H, int W, int64_t ld, T c, uint32_t tiles_x) {
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t ty = tile / tiles_x;
    const uint32_t tx = tile - ty * tiles_x;
    const int lane = threadIdx.x & (kWave - 1);
    const int jb = ((int)tx * kBlock + (int)threadIdx.x) * V;
    const int i0 = 1 + (int)ty * ROWS;       // first output row of the tile
    const int n = min(ROWS, H - 1 - i0);     // output rows in the tile, >= 1 (same for the whole block)
    const int wave_end = (jb - lane * V) + kWave * V;  // one past the wave's last column
    const T* src = in + (int64_t)(i0 - 1) * ld;
    T* dst = out + (int64_t)i0 * ld;
    if (n == ROWS && wave_end <= W)
        sweep_tile<T, V, ROWS, true>(src, dst, n, jb, lane, W, ld, c);
    else
        sweep_tile<T, V, ROWS, false>(src, dst, n, jb, lane, W, ld, c);
}

// END KERNEL SOURCE

// One sweep of each of several independent grids in one launch (the tiles of
// a tiled grid at ghost depth 1). Grid k owns the workgroup tiles [first,
// first + tiles) of the launch; the XCD-aware map deals the launch's tiles as
// for one grid, so each XCD walks a contiguous range of tiles across grids.
// Every grid takes the vector path: 16-byte aligned data, ld a multiple of V.
constexpr int kMaxSweepGrids = 32;

struct SweepGrid {
    const double* in;
    double* out;
    int64_t ld;
    int H, W;
    uint32_t tiles_x, first;
    // mirrors of the edge rows and columns (depth-1 exchange), NULL where none
    double* mn;
    double* ms;
    double* mw;
    double* me;
    int64_t ldw, lde;
};

struct SweepGrids {
    SweepGrid g[kMaxSweepGrids];
    int n;
};

// One tile of a multi-grid sweep that also stores the grid's edge values into
// its neighbours' ghost cells (the depth-1 exchange, GridMirror): the tile
// loop of sweep_tile, with each computed row's values at the first and last
// interior row and column stored a second time, straight from registers.
template <int ROWS, bool FULL>
__device__ __forceinline__ void sweep_tile_mirror(const double* __restrict__ src, double* __restrict__ dst, int n,
                                                  int i0, int jb, int lane, const SweepGrid& gr, double c) {
    constexpr int V = 2;
    const int W = gr.W;
    const int64_t ld = gr.ld;
    double r[ROWS + 2][V];
#pragma unroll
    for (int k = 0; k < ROWS + 2; ++k) {
        if (FULL) {
            typedef typename Vec<double, V>::type VT;
            VT x = *reinterpret_cast<const VT*>(src + (int64_t)k * ld + jb);
#pragma unroll
            for (int e = 0; e < V; ++e) r[k][e] = x[e];
        } else if (k < n + 2) {
            load_vec<double, V>(src + (int64_t)k * ld, jb, W, r[k]);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) r[k][e] = 0.0;
        }
    }
    double el[ROWS], er[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        el[k] = 0.0;
        er[k] = 0.0;
        if (FULL || k < n) {
            const double* row = src + (int64_t)(k + 1) * ld;
            if (lane == 0 && jb > 0 && jb <= W) el[k] = row[jb - 1];
            if (lane == kWave - 1 && jb + V < W) er[k] = row[jb + V];
        }
    }
    // this thread's columns that are the first (west mirror) or last (east mirror) interior column
    const bool col_w = gr.mw != nullptr && jb <= 1 && 1 < jb + V;
    const bool col_e = gr.me != nullptr && jb <= W - 2 && W - 2 < jb + V;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        if (FULL || k < n) {
            double left0 = __shfl_up(r[k + 1][V - 1], 1);
            double rightv = __shfl_down(r[k + 1][0], 1);
            if (lane == 0) left0 = el[k];
            if (lane == kWave - 1) rightv = er[k];
            double o[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const double west = (e == 0) ? left0 : r[k + 1][e > 0 ? e - 1 : 0];
                const double east = (e == V - 1) ? rightv : r[k + 1][e < V - 1 ? e + 1 : 0];
                double t = r[k][e] + r[k + 2][e];  // N + S
                t = t + west;                      // + W
                t = t + east;                      // + E
                o[e] = c * t;
            }
            store_vec<double, V>(dst + (int64_t)k * ld, jb, W, o);
            const int i = i0 + k;
            if ((i == 1 && gr.mn != nullptr) || (i == gr.H - 2 && gr.ms != nullptr)) {  // uniform per row
                double* to = (i == 1 && gr.mn != nullptr) ? gr.mn : gr.ms;
                store_vec<double, V>(to, jb, W, o);
                if (i == 1 && i == gr.H - 2 && gr.mn != nullptr && gr.ms != nullptr) store_vec<double, V>(gr.ms, jb, W, o);
            }
            if (col_w) gr.mw[(int64_t)i * gr.ldw] = o[1 - jb];
            if (col_e) gr.me[(int64_t)i * gr.lde] = o[W - 2 - jb];
        }
    }
}

template <int ROWS>
__global__ __launch_bounds__(kBlock) void sweep_grids_kernel(const SweepGrids grids, double c) {
    constexpr int V = 2;
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    int k = 0;
    while (k + 1 < grids.n && tile >= grids.g[k + 1].first) ++k;
    const SweepGrid& gr = grids.g[k];
    const uint32_t local = tile - gr.first;
    const uint32_t ty = local / gr.tiles_x;
    const uint32_t tx = local - ty * gr.tiles_x;
    const int lane = threadIdx.x & (kWave - 1);
    const int jb = ((int)tx * kBlock + (int)threadIdx.x) * V;
    const int i0 = 1 + (int)ty * ROWS;
    const int n = min(ROWS, gr.H - 1 - i0);
    const int wave_end = (jb - lane * V) + kWave * V;
    const double* src = gr.in + (int64_t)(i0 - 1) * gr.ld;
    double* dst = gr.out + (int64_t)i0 * gr.ld;
    const bool full = n == ROWS && wave_end <= gr.W;
    const bool mirror = gr.mn != nullptr || gr.ms != nullptr || gr.mw != nullptr || gr.me != nullptr;
    if (mirror) {
        if (full)
            sweep_tile_mirror<ROWS, true>(src, dst, n, i0, jb, lane, gr, c);
        else
            sweep_tile_mirror<ROWS, false>(src, dst, n, i0, jb, lane, gr, c);
    } else if (full) {
        sweep_tile<double, V, ROWS, true>(src, dst, n, jb, lane, gr.W, gr.ld, c);
    } else {
        sweep_tile<double, V, ROWS, false>(src, dst, n, jb, lane, gr.W, gr.ld, c);
    }
    // The interior columns past the row's blocks (at most 2, see the launcher) go to the last thread of
    // the row's last block: the same expression, element by element.
    const int covered = (int)gr.tiles_x * kBlock * V;
    if (tx == gr.tiles_x - 1 && threadIdx.x == kBlock - 1 && covered < gr.W - 1) {
        for (int k = 0; k < n; ++k) {
            const int i = i0 + k;
            const double* up = src + (int64_t)k * gr.ld;
            const double* mid = up + gr.ld;
            const double* down = mid + gr.ld;
            for (int j = covered; j < gr.W - 1; ++j) {
                double t = up[j] + down[j];  // N + S
                t = t + mid[j - 1];          // + W
                t = t + mid[j + 1];          // + E
                const double o = c * t;
                dst[(int64_t)k * gr.ld + j] = o;
                if (i == 1 && gr.mn != nullptr) gr.mn[j] = o;
                if (i == gr.H - 2 && gr.ms != nullptr) gr.ms[j] = o;
                if (j == gr.W - 2 && gr.me != nullptr) gr.me[(int64_t)i * gr.lde] = o;
            }
        }
    }
}

// Copy the boundary ring of u0 into d1 and (when not NULL) d2. Needs H, W >= 2.
template <typename T>
__global__ void ring_copy_kernel(const T* __restrict__ u0, T* __restrict__ d1, T* __restrict__ d2,
                                 int H, int W, int64_t ld) {
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
    const T v = u0[off];
    d1[off] = v;
    if (d2 != nullptr) d2[off] = v;
}

// Fill rows [r0, r1) x columns [c0, c1) of a grid with one value.
__global__ void fill_rect_kernel(double* __restrict__ p, int64_t ld, int r0, int r1, int c0, int c1, double v) {
    const int64_t w = c1 - c0;
    const int64_t total = (int64_t)(r1 - r0) * w;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / w;
        const int64_t j = idx - i * w;
        p[(r0 + i) * ld + c0 + j] = v;
    }
}

// Streaming copy of n16 16-byte units between 16-byte aligned buffers (a
// contiguous grid, ld == W): one unit per lane, loaded and stored with the
// non-temporal hint (the copy is read and written once). Measured on MI355X
// at 512 MiB and 2 GiB: 6.45-6.49 TB/s, ahead of 2, 4, 8 or 16 units per
// lane (5.1-5.7 TB/s), of larger workgroups and of grid-stride loops.
constexpr int kCopyBlock = 256;
typedef unsigned int CopyUnit __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kCopyBlock) void copy16_kernel(const CopyUnit* __restrict__ src,
                                                            CopyUnit* __restrict__ dst, int64_t n16) {
    const int64_t k = (int64_t)blockIdx.x * kCopyBlock + threadIdx.x;
    if (k < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

// Bytes past the last whole 16-byte unit of a contiguous copy.
__global__ void copy_tail_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, int n) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

// Copy `bytes` contiguous bytes (both pointers 16-byte aligned).
void launch_copy_contiguous(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    const int64_t n16 = bytes / 16;
    // launches of at most 2^22 workgroups (16 GiB each), inside the 32-bit work-item count
    constexpr int64_t kChunk = ((int64_t)1 << 22) * kCopyBlock;
    for (int64_t off = 0; off < n16; off += kChunk) {
        const int64_t n = std::min(kChunk, n16 - off);
        const int64_t blocks = (n + kCopyBlock - 1) / kCopyBlock;
        copy16_kernel<<<(uint32_t)blocks, kCopyBlock, 0, s>>>(static_cast<const CopyUnit*>(src) + off,
                                                              static_cast<CopyUnit*>(dst) + off, n);
    }
    const int tail = (int)(bytes - n16 * 16);
    if (tail > 0)
        copy_tail_kernel<<<1, 64, 0, s>>>(static_cast<const unsigned char*>(src) + n16 * 16,
                                          static_cast<unsigned char*>(dst) + n16 * 16, tail);
}

// Plain 2-D copy of an H x W grid (degenerate calls: T = 0 or empty interior).
template <typename T>
__global__ void copy_kernel(const T* __restrict__ src, T* __restrict__ dst, int H, int W, int64_t ld) {
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / W;
        const int64_t j = idx - i * W;
        dst[i * ld + j] = src[i * ld + j];
    }
}

// Process-wide tuning settings, read atomically; every accepted value gives
// the same results, so a call racing a setter still computes the method.
std::atomic<int> g_rows_override{0};  // 0: built-in choice; else rows per tile
std::atomic<int> g_schedule{0};       // sweeps per launch of the plain calls: 0 built-in (temporal blocking), 1 single

// Most sweeps per launch the plain calls use when the grid allows temporal
// blocking; the T sweeps are split evenly over ceil(T / levels) launches.
// Measured on MI355X (100 sweeps): FP64 12 (at 4096^2 that is one launch of
// 12 and eight of 11, 3% faster than ten of 10; 12% and 15% faster at 8192^2
// and 16384^2, where HBM alone serves the grid); FP32 8 while one buffer fits
// in half of the 256 MB MALL (4096^2: 8 is 5% faster than 12), else 12
// (8192^2: 24% faster than 8).
template <typename T>
int default_levels(int64_t H, int64_t W) {
    const bool cached = H * W * (int64_t)sizeof(T) <= ((int64_t)128 << 20);  // the pair fits the 256 MiB MALL
    if (sizeof(T) == 8) return cached ? 12 : 14;
    return cached ? 8 : 12;
}

inline sten_status run_tb_any(const double* u0, double* out, double* work, int64_t H, int64_t W, int64_t ld,
                              int32_t T, double c, int32_t levels, hipStream_t s) {
    return run_tb_f64(u0, out, work, H, W, ld, T, c, levels, s);
}
inline sten_status run_tb_any(const float* u0, float* out, float* work, int64_t H, int64_t W, int64_t ld,
                              int32_t T, float c, int32_t levels, hipStream_t s) {
    return run_tb_f32(u0, out, work, H, W, ld, T, c, levels, s);
}

template <typename T, int V, int ROWS>
void launch_sweep_rows(const T* in, T* out, int H, int W, int64_t ld, T c, hipStream_t s) {
    const uint32_t tiles_x = ceil_div(W, (int64_t)kBlock * V);
    const uint32_t tiles_y = ceil_div(H - 2, ROWS);
    sweep_kernel<T, V, ROWS><<<tiles_x * tiles_y, kBlock, 0, s>>>(in, out, H, W, ld, c, tiles_x);
}

template <typename T, int V>
void launch_sweep(const T* in, T* out, int H, int W, int64_t ld, T c, int rows, hipStream_t s) {
    switch (rows) {
        case 16: launch_sweep_rows<T, V, 16>(in, out, H, W, ld, c, s); break;
        case 8: launch_sweep_rows<T, V, 8>(in, out, H, W, ld, c, s); break;
        default: launch_sweep_rows<T, V, 4>(in, out, H, W, ld, c, s); break;
    }
}

template <typename T>
sten_status run_jacobi5(const T* u0, T* out, T* work, int64_t H, int64_t W, int64_t ld, int32_t T_,
                        T c, hipStream_t stream) {
    const bool interior = H >= 3 && W >= 3;
    const bool need_work = interior && T_ >= 2;
    sten_status st = check_grid_args(u0, out, work, need_work, H, W, ld, T_, sizeof(T));
    if (st != STEN_OK || H == 0 || W == 0) return st;
    const int h = (int)H, w = (int)W;
    constexpr int VT = 16 / (int)sizeof(T);
    const int sched = g_schedule.load(std::memory_order_relaxed);
    const int levels = std::min(sched == 0 ? default_levels<T>(H, W) : sched, max_stream_levels<T>());
    if (interior && levels > 1 && T_ >= 2 &&
        ((((uintptr_t)u0 | (uintptr_t)out | (uintptr_t)work) % 16) == 0) && ld % VT == 0) {
        // same bits, fewer passes over HBM: several sweeps per launch
        return run_tb_any(u0, out, work, H, W, ld, T_, c, std::min<int32_t>(levels, T_), stream);
    }
    if (!interior || T_ == 0) {
        const int64_t total = H * W;
        if ((ld == W || H == 1) && (((uintptr_t)u0 | (uintptr_t)out) % 16) == 0) {
            launch_copy_contiguous(u0, out, total * (int64_t)sizeof(T), stream);
        } else {
            const uint32_t blocks = (uint32_t)std::min<int64_t>((total + 255) / 256, 65536);
            copy_kernel<T><<<blocks, 256, 0, stream>>>(u0, out, h, w, ld);
        }
        return check_launch();
    }
    {
        const int64_t nring = 2 * W + 2 * (H - 2);
        ring_copy_kernel<T><<<ceil_div(nring, 256), 256, 0, stream>>>(u0, out, need_work ? work : nullptr,
                                                                       h, w, ld);
    }
    constexpr int VV = 16 / (int)sizeof(T);
    const uintptr_t align_bits = (uintptr_t)u0 | (uintptr_t)out | (need_work ? (uintptr_t)work : 0);
    const bool vec_ok = (align_bits % 16 == 0) && (ld % VV == 0);
    const int rows_set = g_rows_override.load(std::memory_order_relaxed);
    const int rows = rows_set > 0 ? rows_set : 4;
    const T* src = u0;
    for (int32_t k = 1; k <= T_; ++k) {
        T* dst = ((T_ - k) % 2 == 0) ? out : work;
        if (vec_ok)
            launch_sweep<T, VV>(src, dst, h, w, ld, c, rows, stream);
        else
            launch_sweep<T, 1>(src, dst, h, w, ld, c, rows, stream);
        src = dst;
    }
    return check_launch();
}

template <typename T>
sten_status run_sweep_once(const T* src, T* dst, int64_t H, int64_t W, int64_t ld, T c, hipStream_t stream) {
    sten_status st = check_grid_args(src, dst, nullptr, false, H, W, ld, 1, sizeof(T));
    if (st != STEN_OK || H < 3 || W < 3) return st;
    constexpr int VV = 16 / (int)sizeof(T);
    const bool vec_ok = (((uintptr_t)src | (uintptr_t)dst) % 16 == 0) && (ld % VV == 0);
    const int rows_set = g_rows_override.load(std::memory_order_relaxed);
    const int rows = rows_set > 0 ? rows_set : 4;
    if (vec_ok)
        launch_sweep<T, VV>(src, dst, (int)H, (int)W, ld, c, rows, stream);
    else
        launch_sweep<T, 1>(src, dst, (int)H, (int)W, ld, c, rows, stream);
    return check_launch();
}

}  // namespace

void launch_sweep_f64_internal(const double* in, double* out, int H, int W, int64_t ld, double c, hipStream_t s);

// m sweeps ping-ponging between a and b from a (the listing's loop on two
// arrays with equal rings). keep_prev: the first m-1 as blocked launches that
// end in the array iterate m-1 belongs to, then one plain sweep into the other
// array, so both iterates are kept. Otherwise (lands_in_b not null) all m
// sweeps run as the fewest blocked launches, iterate m lands in whichever
// array the last one writes (*lands_in_b: 1 for b, 0 for a), and the other
// array's interior is left unspecified.
sten_status run_chain_f64(double* a, double* b, int64_t H, int64_t W, int64_t ld, int32_t m, double c, bool keep_prev,
                          int32_t* lands_in_b, hipStream_t stream) {
    if (!keep_prev && lands_in_b == nullptr) return STEN_ERR_PTR;
    if (H < 0 || W < 0 || (H > 0 && ld < W) || m < 0 || H > INT32_MAX / 2 || W > INT32_MAX / 2)
        return STEN_ERR_ARG;
    if (!keep_prev) *lands_in_b = m % 2;  // the single-sweep parity, kept for no-op calls
    if (m == 0 || H < 3 || W < 3) return STEN_OK;
    if (a == nullptr || b == nullptr) return STEN_ERR_PTR;
    const size_t span = span_bytes(H, W, ld, sizeof(double));
    if (overlaps(a, span, b, span)) return STEN_ERR_ALIAS;
    if (!is_device_ptr(a) || !is_device_ptr(b)) return STEN_ERR_PTR;
    const int h = (int)H, w = (int)W;
    const int sched = g_schedule.load(std::memory_order_relaxed);
    const int L = sched == 0 ? default_levels<double>(H, W) : sched;
    const bool blocked = L > 1 && (((uintptr_t)a | (uintptr_t)b) % 16) == 0 && ld % 2 == 0 &&
                         W * (int64_t)sizeof(double) < ((int64_t)1 << 30);
    const int n = keep_prev ? m - 1 : m;  // sweeps before the last single one (all of them without keep_prev)
    const double* src = a;
    if (blocked && n >= 2) {
        // k launches; launch j writes b for odd j, a for even j, and the k-th must write the array
        // that holds iterate n (b when n is odd), so k and n have the same parity
        int k = (n + L - 1) / L;
        if (keep_prev && k % 2 != n % 2) ++k;
        else if (!keep_prev) *lands_in_b = k % 2;
        const int base = n / k, extra = n % k;
        for (int j = 1; j <= k; ++j) {
            double* dst = (j % 2) ? b : a;
            const int lev = base + (j <= extra ? 1 : 0);
            if (lev == 1)
                launch_sweep_f64_internal(src, dst, h, w, ld, c, stream);
            else if (!launch_levels_f64(src, dst, h, w, ld, c, lev, stream))
                return STEN_ERR_ARG;  // unreachable: 2 <= lev <= L <= 14 and the rows fit the streaming kernel
            src = dst;
        }
    } else {
        for (int j = 1; j <= n; ++j) {
            double* dst = (j % 2) ? b : a;
            launch_sweep_f64_internal(src, dst, h, w, ld, c, stream);
            src = dst;
        }
    }
    if (keep_prev) launch_sweep_f64_internal(src, src == a ? b : a, h, w, ld, c, stream);
    return check_launch();
}

// One sweep of each of n grids (H, W >= 3; 16-byte aligned, even ld), in
// launches of up to kMaxSweepGrids grids. Returns false, with nothing
// launched, when a grid does not meet the alignment the vector path needs.
bool launch_sweep_grids_f64(const GridView<double>* views, int n, double c, hipStream_t s,
                            const GridMirror* mirrors) {
    constexpr int ROWS = 4;
    for (int k = 0; k < n; ++k)
        if ((((uintptr_t)views[k].in | (uintptr_t)views[k].out) % 16) != 0 || views[k].ld % 2 != 0) return false;
    for (int k0 = 0; k0 < n; k0 += kMaxSweepGrids) {
        SweepGrids args{};
        args.n = std::min(n - k0, kMaxSweepGrids);
        uint32_t first = 0;
        for (int k = 0; k < args.n; ++k) {
            const GridView<double>& v = views[k0 + k];
            SweepGrid& g = args.g[k];
            g.in = v.in;
            g.out = v.out;
            g.ld = v.ld;
            g.H = v.H;
            g.W = v.W;
            // blocks of 512 columns; when the last block would hold at most 2 interior columns (tile
            // views of 2^k + 1 to 2^k + 3 columns), it is dropped and the row's last thread computes them
            g.tiles_x = ceil_div(v.W, (int64_t)kBlock * 2);
            const int64_t tail = (int64_t)(v.W - 1) - (int64_t)(g.tiles_x - 1) * kBlock * 2;
            if (g.tiles_x > 1 && tail <= 2) --g.tiles_x;
            g.first = first;
            if (mirrors != nullptr) {
                const GridMirror& m = mirrors[k0 + k];
                g.mn = m.north;
                g.ms = m.south;
                g.mw = m.west;
                g.me = m.east;
                g.ldw = m.ld_west;
                g.lde = m.ld_east;
            }
            first += g.tiles_x * ceil_div(v.H - 2, ROWS);
        }
        if (first > 0) sweep_grids_kernel<ROWS><<<first, kBlock, 0, s>>>(args, c);
    }
    return true;
}

// FP64 sweep launch for other parts of the library (no argument checks).
void launch_sweep_f64_internal(const double* in, double* out, int H, int W, int64_t ld, double c, hipStream_t s) {
    const bool vec_ok = (((uintptr_t)in | (uintptr_t)out) % 16 == 0) && (ld % 2 == 0);
    const int rows_set = g_rows_override.load(std::memory_order_relaxed);
    const int rows = rows_set > 0 ? rows_set : 4;
    if (vec_ok)
        launch_sweep<double, 2>(in, out, H, W, ld, c, rows, s);
    else
        launch_sweep<double, 1>(in, out, H, W, ld, c, rows, s);
}

// FP32 sweep launch for other parts of the library (no argument checks).
void launch_sweep_f32_internal(const float* in, float* out, int H, int W, int64_t ld, float c, hipStream_t s) {
    const bool vec_ok = (((uintptr_t)in | (uintptr_t)out) % 16 == 0) && (ld % 4 == 0);
    const int rows_set = g_rows_override.load(std::memory_order_relaxed);
    const int rows = rows_set > 0 ? rows_set : 4;
    if (vec_ok)
        launch_sweep<float, 4>(in, out, H, W, ld, c, rows, s);
    else
        launch_sweep<float, 1>(in, out, H, W, ld, c, rows, s);
}

}  // namespace sten

extern "C" {

sten_status sten_fill_rect_f64(double* grid, int64_t H, int64_t W, int64_t ld, int64_t r0, int64_t r1,
                               int64_t c0, int64_t c1, double value, hipStream_t stream) {
    using namespace sten;
    if (H < 0 || W < 0 || (H > 0 && ld < W) || H > INT32_MAX / 2 || W > INT32_MAX / 2) return STEN_ERR_ARG;
    if (r0 < 0 || c0 < 0 || r1 > H || c1 > W || r0 > r1 || c0 > c1) return STEN_ERR_ARG;
    if (r0 == r1 || c0 == c1) return STEN_OK;
    if (grid == nullptr) return STEN_ERR_PTR;
    if (!is_device_ptr(grid)) return STEN_ERR_PTR;
    const int64_t total = (r1 - r0) * (c1 - c0);
    const uint32_t blocks = (uint32_t)std::min<int64_t>((total + 255) / 256, 65536);
    fill_rect_kernel<<<blocks, 256, 0, stream>>>(grid, ld, (int)r0, (int)r1, (int)c0, (int)c1, value);
    return check_launch();
}

sten_status sten_sweep_chain_f64(double* a, double* b, int64_t H, int64_t W, int64_t ld, int32_t m, double c,
                                 hipStream_t stream) {
    return sten::run_chain_f64(a, b, H, W, ld, m, c, true, nullptr, stream);
}

sten_status sten_sweep_chain_last_f64(double* a, double* b, int64_t H, int64_t W, int64_t ld, int32_t m, double c,
                                      int32_t* lands_in_b, hipStream_t stream) {
    return sten::run_chain_f64(a, b, H, W, ld, m, c, false, lands_in_b, stream);
}

sten_status sten_sweep_f64(const double* src, double* dst, int64_t H, int64_t W, int64_t ld, double c,
                           hipStream_t stream) {
    return sten::run_sweep_once<double>(src, dst, H, W, ld, c, stream);
}

sten_status sten_sweep_f32(const float* src, float* dst, int64_t H, int64_t W, int64_t ld, float c,
                           hipStream_t stream) {
    return sten::run_sweep_once<float>(src, dst, H, W, ld, c, stream);
}

sten_status sten_jacobi5_f64(const double* u0, double* out, double* work, int64_t H, int64_t W, int64_t ld,
                             int32_t T, double c, hipStream_t stream) {
    return sten::run_jacobi5<double>(u0, out, work, H, W, ld, T, c, stream);
}

sten_status sten_jacobi5_f32(const float* u0, float* out, float* work, int64_t H, int64_t W, int64_t ld,
                             int32_t T, float c, hipStream_t stream) {
    return sten::run_jacobi5<float>(u0, out, work, H, W, ld, T, c, stream);
}

// Schedule hook: sweeps per launch of the plain calls (1: one sweep per
// launch; 2..12: temporal blocking with that many; 0: built-in).
sten_status sten_tune_schedule(int32_t levels) {
    if (levels < 0 || levels > sten::kMaxStreamLevelsF64) return STEN_ERR_ARG;
    sten::g_schedule = levels;
    return STEN_OK;
}

// Tuning hook: rows per tile of the sweep kernels (4, 8 or 16; 0 restores the
// built-in choice). Returns STEN_ERR_ARG for other values.
sten_status sten_tune_sweep_rows(int32_t rows) {
    if (rows != 0 && rows != 4 && rows != 8 && rows != 16) return STEN_ERR_ARG;
    sten::g_rows_override = rows;
    return STEN_OK;
}

}  // extern "C"
