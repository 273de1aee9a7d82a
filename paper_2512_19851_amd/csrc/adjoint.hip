// Adjoint (reverse mode) of the five-point Jacobi method, an extension beside
// the paper's forward method.
//
// One sweep is a linear map S: ring points are copied, every interior point m
// becomes c * (sum of its four neighbours). Its transpose, in gather form:
//     (S^T g)[n] = [n on the ring] * g[n] + c * sum over the neighbours m of n
//                  that are interior points of g[m]
// for EVERY point n (ring included). T transposed sweeps applied to
// w = dL/du_T give dL/du0. The derivative with respect to c is
//     dL/dc = sum_k sum_{interior m} lambda_{k+1}[m] * nbrsum(u_k)[m],
// lambda_k = dL/du_k, which needs the forward states u_k: one fused kernel per
// transposed step produces lambda_k from lambda_{k+1} and adds that step's
// dot product, accumulated in FP64, into per-workgroup partial sums (each
// workgroup owns a fixed tile, so the sum is deterministic); a single-block
// kernel reduces the partials in a fixed order.
//
// FP32 arithmetic, neighbour terms in the order N, S, W, E (missing or ring
// neighbours contribute an exact zero), then one multiplication by c and, on
// the ring, one addition of the point's own value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "common.hpp"

namespace sten {

// Forward FP32 sweep launcher exported by sweep.hip.
void launch_sweep_f32_internal(const float* in, float* out, int H, int W, int64_t ld, float c, hipStream_t s);

namespace {

constexpr int kAdjBlock = 256;
constexpr int kAdjRows = 8;

__device__ __forceinline__ float interior_val(const float* __restrict__ g, int i, int j, int H, int W, int64_t ld) {
    return (i >= 1 && i <= H - 2 && j >= 1 && j <= W - 2) ? g[(int64_t)i * ld + j] : 0.0f;
}

// Sum of a double over the workgroup (fixed order: lanes by shuffle tree, then waves in order).
__device__ double block_sum(double v) {
    __shared__ double wsum[kAdjBlock / kWave];
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    if (lane == 0) wsum[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += wsum[w];
    __syncthreads();
    return t;
}

// One transposed step: out = S^T g; when u is given, partials[block] (+)=
// sum over this tile's interior points m of g[m] * nbrsum(u)[m].
__global__ __launch_bounds__(kAdjBlock) void adjoint_step_kernel(const float* __restrict__ g,
                                                                 const float* __restrict__ u,
                                                                 float* __restrict__ out,
                                                                 double* __restrict__ partials, int accumulate,
                                                                 int H, int W, int64_t ld, float c,
                                                                 uint32_t tiles_x) {
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t ty = tile / tiles_x;
    const uint32_t tx = tile - ty * tiles_x;
    const int j = (int)tx * kAdjBlock + (int)threadIdx.x;
    const int i0 = (int)ty * kAdjRows;
    double acc = 0.0;
    if (j < W) {
        const bool ring_col = (j == 0 || j == W - 1);
#pragma unroll
        for (int r = 0; r < kAdjRows; ++r) {
            const int i = i0 + r;
            if (i < H) {
                const float tn = interior_val(g, i - 1, j, H, W, ld);
                const float ts = interior_val(g, i + 1, j, H, W, ld);
                const float tw = interior_val(g, i, j - 1, H, W, ld);
                const float te = interior_val(g, i, j + 1, H, W, ld);
                float s = tn + ts;
                s = s + tw;
                s = s + te;
                const float gc = g[(int64_t)i * ld + j];
                const bool ring = ring_col || i == 0 || i == H - 1;
                const float cs = c * s;
                out[(int64_t)i * ld + j] = ring ? gc + cs : cs;
                if (u != nullptr && !ring) {
                    const int64_t q = (int64_t)i * ld + j;
                    float ns = u[q - ld] + u[q + ld];
                    ns = ns + u[q - 1];
                    ns = ns + u[q + 1];
                    acc += (double)gc * (double)ns;
                }
            }
        }
    }
    if (partials != nullptr) {
        const double t = block_sum(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = accumulate ? partials[blockIdx.x] + t : t;
    }
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// Fixed-order sum of n doubles by one workgroup: thread t sums t, t+B, ...;
// then a tree over threads.
__global__ __launch_bounds__(kAdjBlock) void reduce_f64_kernel(const double* __restrict__ p, int64_t n,
                                                               double* __restrict__ out) {
    double v = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) v += p[k];
    const double t = block_sum(v);
    if (threadIdx.x == 0) *out = t;
}

__global__ void copy_f32_kernel(const float* __restrict__ src, float* __restrict__ dst, int H, int W, int64_t ld) {
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / W;
        const int64_t j = idx - i * W;
        dst[i * ld + j] = src[i * ld + j];
    }
}

// Copy u0's ring into planes 1..nplanes-1 of `states` (plane stride `pstride` elements).
__global__ void ring_to_planes_kernel(const float* __restrict__ u0, float* __restrict__ states, int nplanes,
                                      int64_t pstride, int H, int W, int64_t ld) {
    const int64_t nring = 2 * (int64_t)W + 2 * (int64_t)(H - 2);
    const int64_t total = nring * (nplanes - 1);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = 1 + idx / nring;
        const int64_t r = idx - (p - 1) * nring;
        int i, j;
        if (r < W) {
            i = 0;
            j = (int)r;
        } else if (r < 2 * (int64_t)W) {
            i = H - 1;
            j = (int)(r - W);
        } else {
            const int64_t k = r - 2 * (int64_t)W;
            i = 1 + (int)(k >> 1);
            j = (k & 1) ? W - 1 : 0;
        }
        const int64_t off = (int64_t)i * ld + j;
        states[p * pstride + off] = u0[off];
    }
}

inline uint32_t grid_for(int64_t total) {
    return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

inline uint32_t adj_tiles_x(int64_t W) { return ceil_div(W, kAdjBlock); }
inline uint32_t adj_blocks(int64_t H, int64_t W) { return adj_tiles_x(W) * ceil_div(H, kAdjRows); }

sten_status check_dims(int64_t H, int64_t W, int64_t ld, int32_t T) {
    if (H < 0 || W < 0 || T < 0) return STEN_ERR_ARG;
    if (H > 0 && ld < W) return STEN_ERR_ARG;
    if (H > INT32_MAX - 2 || W > INT32_MAX - 2) return STEN_ERR_ARG;
    return STEN_OK;
}

// The transposed steps of one segment; `partials` (when not NULL) holds at
// least adj_blocks(H, W) doubles of device memory, queried here when
// check_partials is set (the library's own static buffer is not).
sten_status adjoint_seg(const float* lam_in, const float* states, int32_t nsteps, float* lam_out, float* work,
                        double* partials, bool check_partials, int32_t reset, int64_t H, int64_t W, int64_t ld,
                        float c, hipStream_t stream) {
    sten_status st = check_dims(H, W, ld, nsteps);
    if (st != STEN_OK || H == 0 || W == 0) return st;
    if (lam_in == nullptr || lam_out == nullptr) return STEN_ERR_PTR;
    const bool need_work = nsteps >= 2;
    if (need_work && work == nullptr) return STEN_ERR_PTR;
    const size_t gb = span_bytes(H, W, ld, 4);
    if (overlaps(lam_in, gb, lam_out, gb)) return STEN_ERR_ALIAS;
    if (need_work && (overlaps(lam_in, gb, work, gb) || overlaps(lam_out, gb, work, gb))) return STEN_ERR_ALIAS;
    const int64_t pstride = H * ld;
    if (states != nullptr && nsteps > 0) {
        const size_t sb = (size_t)(nsteps - 1) * pstride * 4 + gb;
        if (overlaps(states, sb, lam_out, gb) || (need_work && overlaps(states, sb, work, gb)))
            return STEN_ERR_ALIAS;
    }
    if (!is_device_ptr(lam_in) || !is_device_ptr(lam_out) || (need_work && !is_device_ptr(work)))
        return STEN_ERR_PTR;
    if (states != nullptr && !is_device_ptr(states)) return STEN_ERR_PTR;
    if (check_partials && partials != nullptr && !is_device_ptr(partials)) return STEN_ERR_PTR;
    const int h = (int)H, w = (int)W;
    const uint32_t nb = adj_blocks(H, W);
    const bool degenerate = (H < 3 || W < 3);
    if (partials != nullptr && reset && (nsteps == 0 || degenerate || states == nullptr))
        fill_f64_kernel<<<grid_for(nb), 256, 0, stream>>>(partials, nb, 0.0);
    if (nsteps == 0 || degenerate) {
        copy_f32_kernel<<<grid_for(H * W), 256, 0, stream>>>(lam_in, lam_out, h, w, ld);
        return check_launch();
    }
    const float* src = lam_in;
    for (int32_t s = 1; s <= nsteps; ++s) {
        float* dst = ((nsteps - s) % 2 == 0) ? lam_out : work;
        const float* u = states != nullptr ? states + (int64_t)(nsteps - s) * pstride : nullptr;
        const int acc = (s == 1 && reset) ? 0 : 1;
        adjoint_step_kernel<<<nb, kAdjBlock, 0, stream>>>(src, u, dst, u != nullptr ? partials : nullptr, acc, h, w,
                                                         ld, c, adj_tiles_x(W));
        src = dst;
    }
    return check_launch();
}

// FP64 partial sums of sten_jacobi5_adjoint_f32_seg_noalloc, one per
// workgroup of a transposed step, in a per-device static buffer, so that the
// call allocates nothing. Every call on a device shares that device's buffer.
constexpr size_t kStaticPartials = (size_t)1 << 20;  // 8 MiB per device
static __device__ __align__(256) double scratch[kStaticPartials];

// Device address of `scratch` on each device, taken once per device with that
// device current (in host code the array's name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

sten_status scratch_partials(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= kMaxDevices) return STEN_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return STEN_OK;
}

}  // namespace
}  // namespace sten

extern "C" {

size_t sten_adjoint_partials_len(int64_t H, int64_t W) {
    if (H <= 0 || W <= 0) return 1;
    return (size_t)sten::adj_blocks(H, W);
}

sten_status sten_jacobi5_f32_states(const float* u0, float* states, int64_t H, int64_t W, int64_t ld, int32_t T,
                                    float c, hipStream_t stream) {
    using namespace sten;
    sten_status st = check_dims(H, W, ld, T);
    if (st != STEN_OK || H == 0 || W == 0) return st;
    if (u0 == nullptr || states == nullptr) return STEN_ERR_PTR;
    const int64_t pstride = H * ld;
    const size_t gb = span_bytes(H, W, ld, 4);
    const size_t sb = (size_t)T * pstride * 4 + gb;
    if (overlaps(u0, gb, states, sb)) return STEN_ERR_ALIAS;
    if (!is_device_ptr(u0) || !is_device_ptr(states)) return STEN_ERR_PTR;
    const int h = (int)H, w = (int)W;
    copy_f32_kernel<<<grid_for(H * W), 256, 0, stream>>>(u0, states, h, w, ld);
    if (H >= 3 && W >= 3) {
        if (T > 0) {
            const int64_t nring = 2 * W + 2 * (H - 2);
            ring_to_planes_kernel<<<grid_for(nring * T), 256, 0, stream>>>(u0, states, T + 1, pstride, h, w, ld);
        }
        for (int32_t k = 1; k <= T; ++k)
            launch_sweep_f32_internal(states + (k - 1) * pstride, states + k * pstride, h, w, ld, c, stream);
    } else {
        for (int32_t k = 1; k <= T; ++k)
            copy_f32_kernel<<<grid_for(H * W), 256, 0, stream>>>(u0, states + k * pstride, h, w, ld);
    }
    return check_launch();
}

sten_status sten_jacobi5_adjoint_f32_seg(const float* lam_in, const float* states, int32_t nsteps, float* lam_out,
                                         float* work, double* partials, int32_t reset, int64_t H, int64_t W,
                                         int64_t ld, float c, hipStream_t stream) {
    return sten::adjoint_seg(lam_in, states, nsteps, lam_out, work, partials, true, reset, H, W, ld, c, stream);
}

sten_status sten_jacobi5_adjoint_f32(const float* gout, float* gin, float* work, int64_t H, int64_t W, int64_t ld,
                                     int32_t T, float c, hipStream_t stream) {
    return sten_jacobi5_adjoint_f32_seg(gout, nullptr, T, gin, work, nullptr, 0, H, W, ld, c, stream);
}

sten_status sten_reduce_f64(const double* partials, int64_t n, double* out, hipStream_t stream) {
    using namespace sten;
    if (n < 0) return STEN_ERR_ARG;
    if (partials == nullptr || out == nullptr) return STEN_ERR_PTR;
    if (!is_device_ptr(partials) || !is_device_ptr(out)) return STEN_ERR_PTR;
    reduce_f64_kernel<<<1, kAdjBlock, 0, stream>>>(partials, n, out);
    return check_launch();
}

sten_status sten_jacobi5_adjoint_f32_seg_noalloc(const float* lam_in, const float* states, int32_t nsteps,
                                                 float* lam_out, float* work, int32_t reset, double* dLdc,
                                                 int64_t H, int64_t W, int64_t ld, float c, hipStream_t stream) {
    using namespace sten;
    sten_status st = check_dims(H, W, ld, nsteps);
    if (st != STEN_OK) return st;
    if (H == 0 || W == 0) return STEN_OK;
    if (sten_adjoint_partials_len(H, W) > kStaticPartials) return STEN_ERR_WORKSPACE;
    if (dLdc != nullptr) {
        const size_t gb = span_bytes(H, W, ld, 4);
        if (overlaps(dLdc, sizeof(double), lam_out, gb) || (nsteps >= 2 && overlaps(dLdc, sizeof(double), work, gb)))
            return STEN_ERR_ALIAS;
        if (!is_device_ptr(dLdc)) return STEN_ERR_PTR;
    }
    double* partials = nullptr;
    if ((st = scratch_partials(&partials)) != STEN_OK) return st;
    st = adjoint_seg(lam_in, states, nsteps, lam_out, work, partials, false, reset, H, W, ld, c, stream);
    if (st != STEN_OK || dLdc == nullptr) return st;
    reduce_f64_kernel<<<1, kAdjBlock, 0, stream>>>(partials, (int64_t)sten_adjoint_partials_len(H, W), dLdc);
    return check_launch();
}

}  // extern "C"
