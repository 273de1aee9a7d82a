// Batched form of the five-point Jacobi method: many independent grids of
// uneven size, each iterated T times, in ONE persistent kernel launch.
//
// The paper runs one generated kernel per chare per iteration, with many
// chares per GPU (over-decomposition, Section III-C). For small grids that
// model is launch-bound: 1024 grids x T sweeps would be 1024*T launches. Here
// every workgroup instead pulls whole grids from an atomic work queue and runs
// all T sweeps of a grid itself, separated only by workgroup barriers:
//  * grids whose two ping-pong buffers fit the workgroup's LDS budget are
//    loaded once, swept T times entirely in LDS and written back once;
//  * larger grids sweep between the caller's out/work buffers in global
//    memory; their working set stays in L2 / Infinity Cache across sweeps.
// The host plan sorts grids by estimated cost (largest first) so the dynamic
// queue performs longest-processing-time list scheduling, and uploads the
// sorted descriptors to caller-provided device workspace. A run is two kernel
// launches (queue reset + persistent sweep kernel) and no allocation or
// memset, so it can be captured in a HIP graph.
//
// The arithmetic per point is the listing's (Section III-A) in FP32,
// c * (((N + S) + W) + E), bit-identical to the single-grid FP32 path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace sten {
namespace {

enum : int32_t { MODE_COPY = 0, MODE_LDS = 1, MODE_GLOBAL = 2, MODE_REG = 3 };


struct alignas(16) Desc {
    const float* u0;
    float* out;
    float* work;
    int32_t H, W, ld, mode;
};

constexpr size_t kCounterBytes = 256;

// Interior point p (0-based, row-major over the (H-2) x (W-2) interior) of a
// grid with interior width w: advance by `step` points at a time without
// dividing in the loop.
struct Walker {
    int i, j;       // current point (grid coordinates, 1-based interior)
    int di, dj;     // step as whole rows + remaining columns
    int w;          // interior width
    __device__ void init(int p, int step, int width) {
        w = width;
        i = 1 + p / w;
        j = 1 + p % w;
        di = step / w;
        dj = step % w;
    }
    __device__ void next() {
        i += di;
        j += dj;
        if (j > w) {
            j -= w;
            i += 1;
        }
    }
};

__device__ __forceinline__ float stencil(float n, float s, float w, float e, float c) {
    float t = n + s;
    t = t + w;
    t = t + e;
    return c * t;
}

__device__ __forceinline__ void run_copy(const Desc& d) {
    const int n = d.H * d.W;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const int i = p / d.W;
        const int j = p - i * d.W;
        d.out[(int64_t)i * d.ld + j] = d.u0[(int64_t)i * d.ld + j];
    }
}

// T sweeps with both buffers in LDS (packed rows, stride W).
__device__ __forceinline__ void run_lds(const Desc& d, int T, float c, float* lds) {
    const int H = d.H, W = d.W;
    const int n = H * W;
    float* A = lds;
    float* B = lds + n;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const int i = p / W;
        const int j = p - i * W;
        const float v = d.u0[(int64_t)i * d.ld + j];
        A[p] = v;
        B[p] = v;
    }
    __syncthreads();
    const int w = W - 2;
    const int m = (H - 2) * w;
    for (int t = 0; t < T; ++t) {
        Walker it;
        it.init(threadIdx.x, blockDim.x, w);
        for (int p = threadIdx.x; p < m; p += blockDim.x) {
            const int q = it.i * W + it.j;
            B[q] = stencil(A[q - W], A[q + W], A[q - 1], A[q + 1], c);
            it.next();
        }
        __syncthreads();
        float* tmp = A;
        A = B;
        B = tmp;
    }
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const int i = p / W;
        const int j = p - i * W;
        d.out[(int64_t)i * d.ld + j] = A[p];
    }
}

// T sweeps between the grid's out and work buffers in global memory.
__device__ __forceinline__ void run_global(const Desc& d, int T, float c) {
    const int H = d.H, W = d.W;
    const int64_t ld = d.ld;
    // ring of u0 into out (and work when it is written)
    const int nring = 2 * W + 2 * (H - 2);
    for (int r = threadIdx.x; r < nring; r += blockDim.x) {
        int i, j;
        if (r < W) {
            i = 0;
            j = r;
        } else if (r < 2 * W) {
            i = H - 1;
            j = r - W;
        } else {
            const int k = r - 2 * W;
            i = 1 + (k >> 1);
            j = (k & 1) ? W - 1 : 0;
        }
        const float v = d.u0[i * ld + j];
        d.out[i * ld + j] = v;
        if (T >= 2) d.work[i * ld + j] = v;
    }
    const int w = W - 2;
    const int m = (H - 2) * w;
    const float* src = d.u0;
    for (int k = 1; k <= T; ++k) {
        float* dst = ((T - k) % 2 == 0) ? d.out : d.work;
        Walker it;
        it.init(threadIdx.x, blockDim.x, w);
        for (int p = threadIdx.x; p < m; p += blockDim.x) {
            const int64_t q = (int64_t)it.i * ld + it.j;
            dst[q] = stencil(src[q - ld], src[q + ld], src[q - 1], src[q + 1], c);
            it.next();
        }
        __syncthreads();  // this sweep's writes are visible to the whole workgroup before the next reads
        src = dst;
    }
}

// Register-resident sweeps: the whole grid lives in registers for all T sweeps.
// Each lane holds V consecutive columns (64*V >= W, so one wave spans a whole
// row) of R consecutive rows; wave w holds rows [w*R, w*R + R). Up/down
// neighbours come from the lane's own registers; left/right neighbours from
// its own registers or, for its first and last column, from the adjacent
// lane by a DPP wave shift (the last column of the grid is the ring, so no
// wave ever needs a column from another wave). Only each wave's first and
// last row cross to other waves, through a double-buffered LDS area (parity =
// sweep mod 2), so one workgroup barrier per sweep suffices. Rows are updated
// in order with the previous row's old values kept in `prev` (in-place
// rolling update). Rows past the grid are dummies: loaded as 0, never
// computed, never stored.
constexpr int kRegMaxV = 4;   // columns per lane: a row of up to 256 columns per wave
constexpr int kRegMaxR = 16;  // rows per lane

struct RegShape {
    int V, R;  // columns and rows per lane (0: the grid does not fit)
};

// The smallest lane tile that covers the grid: V = ceil(W / 64) columns and
// R = ceil(H / waves) rows per lane (every row count 1..16 has a kernel
// variant). Every lane computes its whole tile each
// sweep (points past the grid are computed and dropped), so sweep time
// follows V * R, not the grid's point count: a tight tile keeps a 130 x 130
// grid from costing as much as a 256 x 256 one.
__device__ __host__ inline RegShape reg_shape(int H, int W, int block) {
    const int nw = block / 64;
    RegShape s{0, 0};
    const int v = (W + 63) / 64;
    const int r = (H + nw - 1) / nw;
    if (v < 1 || v > kRegMaxV || r < 1 || r > kRegMaxR) return s;
    s.V = v;
    s.R = r;
    return s;
}

// LDS floats of the row exchange area (both parities, first and last row of every wave).
__device__ __host__ inline int reg_lds_floats(const RegShape& s, int block) { return 2 * 2 * (block / 64) * 64 * s.V; }

// DPP wave shifts with bound control set: the lane without a source (lane 0,
// resp. 63) reads 0, so no register has to be cleared first and the shift can
// fold into the add that consumes it.
__device__ __forceinline__ float dpp_from_lower_lane(float v) {  // lane l receives lane l-1
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_from_upper_lane(float v) {  // lane l receives lane l+1
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

template <int V, int R>
__device__ __forceinline__ void run_reg(const Desc& d, int T, float c, float* lds) {
    const int H = d.H, W = d.W;
    const int64_t ld = d.ld;
    const int nw = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int i0 = wave * R;
    const int j0 = lane * V;
    const int rowf = 64 * V;       // floats of one published row
    const int half = 2 * nw * rowf;
    // published slots: first row of wave w at [w*rowf], last row at [(nw + w)*rowf]
    const int o_first = wave * rowf + j0;
    const int o_last = (nw + wave) * rowf + j0;
    const int o_above = (nw + wave - 1) * rowf + j0;  // last row of the wave above
    const int o_below = (wave + 1) * rowf + j0;       // first row of the wave below
    bool col_in[V];
#pragma unroll
    for (int e = 0; e < V; ++e) col_in[e] = (j0 + e >= 1) && (j0 + e <= W - 2);

    float v[R][V];
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e)
            v[k][e] = (i0 + k < H && j0 + e < W) ? d.u0[(int64_t)(i0 + k) * ld + j0 + e] : 0.0f;
#pragma unroll
    for (int e = 0; e < V; ++e) {
        lds[o_first + e] = v[0][e];
        lds[o_last + e] = v[R - 1][e];
    }
    __syncthreads();
    // One sweep in either row order. Downward, each row's new values replace its
    // old ones once the next row has read them (kept in `prev`); upward, the same
    // with `next`. Two sweeps in opposite orders per loop iteration let every
    // loop-carried row end in the register it started in (a single direction
    // shifts the rows by one register row per sweep, paid for with copies).
    auto sweep = [&](const float* cur_h, float* nxt_h, auto down) {
        // Re-read the wave's first row each sweep, so that the R x V point masks below are
        // formed in the loop by scalar instructions: hoisted out of it, they need more
        // SGPRs than there are and spill to VGPR lanes that every sweep reads back.
        int i0_t = i0;
        asm volatile("" : "+s"(i0_t));
        float above[V], below[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            above[e] = (wave > 0) ? cur_h[o_above + e] : 0.0f;
            below[e] = (wave + 1 < nw) ? cur_h[o_below + e] : 0.0f;
        }
        float carry[V];  // old values of the row just updated (above it when downward, below when upward)
#pragma unroll
        for (int e = 0; e < V; ++e) carry[e] = down ? above[e] : below[e];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int k = down ? q : R - 1 - q;
            const int i = i0_t + k;
            const bool row_in = (i >= 1) && (i <= H - 2);
            const float lft = dpp_from_lower_lane(v[k][V - 1]);  // column j0 - 1
            const float rgt = dpp_from_upper_lane(v[k][0]);      // column j0 + V
            float nv[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                float up, dn;
                if (down) {
                    up = carry[e];
                    dn = (k == R - 1) ? below[e] : v[k + 1 < R ? k + 1 : k][e];
                } else {
                    up = (k == 0) ? above[e] : v[k > 0 ? k - 1 : 0][e];
                    dn = carry[e];
                }
                const float w_ = (e == 0) ? lft : v[k][e > 0 ? e - 1 : 0];
                const float e_ = (e == V - 1) ? rgt : v[k][e < V - 1 ? e + 1 : 0];
                nv[e] = (row_in && col_in[e]) ? stencil(up, dn, w_, e_, c) : v[k][e];
            }
#pragma unroll
            for (int e = 0; e < V; ++e) {
                carry[e] = v[k][e];
                v[k][e] = nv[e];
            }
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            nxt_h[o_first + e] = v[0][e];
            nxt_h[o_last + e] = v[R - 1][e];
        }
        __syncthreads();
    };
    int t = 0;
    for (; t + 1 < T; t += 2) {
        sweep(lds, lds + half, std::true_type{});
        sweep(lds + half, lds, std::false_type{});
    }
    if (t < T) sweep(lds, lds + half, std::true_type{});
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (i0 + k < H && j0 + e < W) d.out[(int64_t)(i0 + k) * ld + j0 + e] = v[k][e];
}

__device__ __forceinline__ void run_reg_any(const Desc& d, int T, float c, float* lds, int code) {
    // code = V * 32 + R
    switch (code) {
#define STEN_REG_CASE(V_, R_) \
    case V_ * 32 + R_: run_reg<V_, R_>(d, T, c, lds); break;
#define STEN_REG_ROWS(V_)                                                                                     \
    STEN_REG_CASE(V_, 1) STEN_REG_CASE(V_, 2) STEN_REG_CASE(V_, 3) STEN_REG_CASE(V_, 4) STEN_REG_CASE(V_, 5)   \
    STEN_REG_CASE(V_, 6) STEN_REG_CASE(V_, 7) STEN_REG_CASE(V_, 8) STEN_REG_CASE(V_, 9) STEN_REG_CASE(V_, 10)   \
    STEN_REG_CASE(V_, 11) STEN_REG_CASE(V_, 12) STEN_REG_CASE(V_, 13) STEN_REG_CASE(V_, 14) STEN_REG_CASE(V_, 15) \
    STEN_REG_CASE(V_, 16)
        STEN_REG_ROWS(1) STEN_REG_ROWS(2) STEN_REG_ROWS(3) STEN_REG_ROWS(4)
#undef STEN_REG_ROWS
#undef STEN_REG_CASE
        default: break;
    }
}

__global__ void batch_reset_kernel(uint32_t* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

__global__ void batch_kernel(const Desc* __restrict__ descs, uint32_t* __restrict__ counter, int count, int T,
                             float c) {
    extern __shared__ float lds[];
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= count) break;  // every workgroup reaches this once the queue is drained
        const Desc d = descs[idx];
        if ((d.mode & 0xFF) == MODE_REG)
            run_reg_any(d, T, c, lds, d.mode >> 8);
        else if (d.mode == MODE_LDS)
            run_lds(d, T, c, lds);
        else if (d.mode == MODE_GLOBAL)
            run_global(d, T, c);
        else
            run_copy(d);
        __syncthreads();
    }
}

struct Config {
    int block = 1024;
    int lds_bytes = 160 * 1024;  // clamped to the device limit at plan time
    int wg_per_cu = 1;
    int use_reg = 1;             // register-resident mode for grids that fit
};

}  // namespace
}  // namespace sten

struct sten_batch_plan_s {
    int count = 0;
    int T = 0;
    float c = 0.25f;
    sten::Config cfg;
    int grid = 0;
    int n_lds = 0, n_global = 0, n_copy = 0, n_reg = 0;
    sten::Desc* d_descs = nullptr;
    uint32_t* d_counter = nullptr;
    std::vector<sten::Desc> h_descs;
    std::vector<sten_inst> h_insts;  // caller order, kept for re-planning
};

namespace sten {
namespace {

std::mutex g_cache_mutex;

// Cache key: T and a coarse histogram of grid sizes (enough to separate workloads).
std::string batch_key(const sten_inst* insts, int count, int T) {
    uint64_t h = 1469598103934665603ull;
    int64_t total = 0;
    for (int k = 0; k < count; ++k) {
        const uint64_t v = ((uint64_t)(uint32_t)insts[k].H << 32) | (uint32_t)insts[k].W;
        h = (h ^ v) * 1099511628211ull;
        total += (int64_t)insts[k].H * insts[k].W;
    }
    std::ostringstream os;
    os << "count=" << count << ";T=" << T << ";points=" << total << ";shape_hash=" << std::hex << h;
    return os.str();
}

bool cache_lookup(const char* path, const std::string& key, Config& cfg) {
    if (path == nullptr) return false;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {  // later lines win
        const size_t sp = line.find(' ');
        if (sp == std::string::npos || line.substr(0, sp) != key) continue;
        Config c2;
        if (sscanf(line.c_str() + sp + 1, "block=%d lds_bytes=%d wg_per_cu=%d use_reg=%d", &c2.block,
                   &c2.lds_bytes, &c2.wg_per_cu, &c2.use_reg) == 4) {
            cfg = c2;
            found = true;
        }
    }
    return found;
}

bool cache_store(const char* path, const std::string& key, const Config& cfg, float us) {
    if (path == nullptr) return false;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    std::ofstream f(path, std::ios::app);
    if (!f) return false;
    f << key << " block=" << cfg.block << " lds_bytes=" << cfg.lds_bytes << " wg_per_cu=" << cfg.wg_per_cu
      << " use_reg=" << cfg.use_reg << " us=" << us << "\n";
    return (bool)f;
}

int device_lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 64 * 1024;
    return v;
}

int device_cus() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return v;
}

// Static LDS used by the kernel itself (the queue index), kept out of the budget.
constexpr int kStaticLds = 64;

sten_status validate_insts(const sten_inst* insts, int count) {
    for (int k = 0; k < count; ++k) {
        const sten_inst& s = insts[k];
        if (s.H < 0 || s.W < 0) return STEN_ERR_ARG;
        if (s.H > 0 && s.ld < s.W) return STEN_ERR_ARG;
        if ((int64_t)s.H * s.ld > INT32_MAX) return STEN_ERR_ARG;
        if (s.H == 0 || s.W == 0) continue;
        if (s.u0 == nullptr || s.out == nullptr) return STEN_ERR_PTR;
        const size_t nb = span_bytes(s.H, s.W, s.ld, sizeof(float));
        if (overlaps(s.u0, nb, s.out, nb)) return STEN_ERR_ALIAS;
        if (s.work != nullptr && (overlaps(s.u0, nb, s.work, nb) || overlaps(s.out, nb, s.work, nb)))
            return STEN_ERR_ALIAS;
    }
    return STEN_OK;
}

// Classify, cost and sort; fills plan->h_descs and the class counts.
void build_descs(sten_batch_plan_s* p) {
    const int lds_floats = (p->cfg.lds_bytes - kStaticLds) / (int)sizeof(float);
    struct Item {
        Desc d;
        double cost;
    };
    std::vector<Item> items;
    items.reserve(p->count);
    p->n_lds = p->n_global = p->n_copy = p->n_reg = 0;
    for (const sten_inst& s : p->h_insts) {
        if (s.H == 0 || s.W == 0) continue;
        Desc d{s.u0, s.out, s.work, s.H, s.W, s.ld, MODE_COPY};
        double cost = (double)s.H * s.W;
        if (s.H >= 3 && s.W >= 3 && p->T > 0) {
            const double pts = (double)(s.H - 2) * (s.W - 2) * p->T;
            const RegShape rs = reg_shape(s.H, s.W, p->cfg.block);
            if (p->cfg.use_reg && rs.V > 0 && reg_lds_floats(rs, p->cfg.block) <= lds_floats) {
                d.mode = MODE_REG | ((rs.V * 32 + rs.R) << 8);
                cost = 0.3 * p->T * (double)(p->cfg.block / 64) * rs.R * 64 * rs.V;  // lane-points swept
            } else if (2 * s.H * s.W <= lds_floats) {
                d.mode = MODE_LDS;
                cost = pts + 2.0 * s.H * s.W;
            } else {
                d.mode = MODE_GLOBAL;
                cost = 2.5 * pts;  // global sweeps move about 2.5x the bytes of LDS sweeps per point
            }
        }
        if ((d.mode & 0xFF) == MODE_REG) ++p->n_reg;
        else if (d.mode == MODE_LDS) ++p->n_lds;
        else if (d.mode == MODE_GLOBAL) ++p->n_global;
        else ++p->n_copy;
        items.push_back({d, cost});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    p->h_descs.clear();
    for (const Item& it : items) p->h_descs.push_back(it.d);
}

// A grid swept in global memory with T >= 2 ping-pongs through its `work`
// buffer, so that buffer must exist. Which grids land in global mode depends
// on the configuration (LDS budget, block, register mode), so this is checked
// after every classification, before anything reaches the device.
sten_status check_global_work(const sten_batch_plan_s* p) {
    if (p->T < 2) return STEN_OK;
    for (const Desc& d : p->h_descs)
        if (d.mode == MODE_GLOBAL && (d.work == nullptr || !is_device_ptr(d.work))) return STEN_ERR_PTR;
    return STEN_OK;
}

// Classify under p->cfg, check the classification and upload the descriptors.
// On STEN_ERR_PTR nothing has been sent to the device: the previously
// uploaded descriptors (if any) are unchanged, but h_descs and the class
// counts describe the rejected configuration until the caller finalizes again.
sten_status finalize_plan(sten_batch_plan_s* p, hipStream_t stream) {
    const int limit = device_lds_limit();
    p->cfg.lds_bytes = std::min(p->cfg.lds_bytes, limit);
    p->cfg.lds_bytes = std::max(p->cfg.lds_bytes, kStaticLds + 16);
    build_descs(p);
    sten_status st = check_global_work(p);
    if (st != STEN_OK) return st;
    p->grid = std::max(1, device_cus() * std::max(1, p->cfg.wg_per_cu));
    const size_t dyn = (size_t)(p->cfg.lds_bytes - kStaticLds);
    hipError_t e = hipFuncSetAttribute((const void*)batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)dyn);
    if (e != hipSuccess) return hip_fail(e);
    if (!p->h_descs.empty()) {
        e = hipMemcpyAsync(p->d_descs, p->h_descs.data(), p->h_descs.size() * sizeof(Desc), hipMemcpyHostToDevice,
                           stream);
        if (e != hipSuccess) return hip_fail(e);
    }
    return STEN_OK;
}

sten_status launch_plan(const sten_batch_plan_s* p, hipStream_t stream) {
    const int n = (int)p->h_descs.size();
    if (n == 0) return STEN_OK;
    batch_reset_kernel<<<1, 64, 0, stream>>>(p->d_counter);
    const size_t dyn = (size_t)(p->cfg.lds_bytes - kStaticLds);
    batch_kernel<<<p->grid, p->cfg.block, dyn, stream>>>(p->d_descs, p->d_counter, n, p->T, p->c);
    return check_launch();
}

}  // namespace
}  // namespace sten

extern "C" {

size_t sten_batch_workspace_bytes(int32_t count) {
    if (count < 0) return 0;
    return sten::kCounterBytes + (size_t)count * sizeof(sten::Desc);
}

sten_status sten_batch_plan(const sten_inst* insts, int32_t count, int32_t T, float c, const char* tune_cache_path,
                            void* dev_ws, size_t ws_bytes, sten_batch_handle* plan, hipStream_t stream) {
    using namespace sten;
    if (plan == nullptr) return STEN_ERR_ARG;
    *plan = nullptr;
    if (count < 0 || T < 0) return STEN_ERR_ARG;
    if (count > 0 && insts == nullptr) return STEN_ERR_PTR;
    if (dev_ws == nullptr) return STEN_ERR_PTR;
    if ((uintptr_t)dev_ws % 256 != 0) return STEN_ERR_ARG;
    if (ws_bytes < sten_batch_workspace_bytes(count)) return STEN_ERR_WORKSPACE;
    sten_status st = validate_insts(insts, count);
    if (st != STEN_OK) return st;
    if (!is_device_ptr(dev_ws)) return STEN_ERR_PTR;
    for (int k = 0; k < count; ++k) {
        const sten_inst& s = insts[k];
        if (s.H == 0 || s.W == 0) continue;
        if (!is_device_ptr(s.u0) || !is_device_ptr(s.out)) return STEN_ERR_PTR;
    }
    auto* p = new sten_batch_plan_s();
    p->count = count;
    p->T = T;
    p->c = c;
    p->h_insts.assign(insts, insts + count);
    p->d_counter = (uint32_t*)dev_ws;
    p->d_descs = (Desc*)((char*)dev_ws + kCounterBytes);
    Config cfg;
    if (!cache_lookup(tune_cache_path, batch_key(insts, count, T), cfg)) cfg = Config{};
    p->cfg = cfg;
    st = finalize_plan(p, stream);  // rejects a global-mode grid without `work` (T >= 2)
    if (st != STEN_OK) {
        delete p;
        return st;
    }
    *plan = p;
    return STEN_OK;
}

sten_status sten_batch_run(sten_batch_handle plan, hipStream_t stream) {
    if (plan == nullptr) return STEN_ERR_ARG;
    return sten::launch_plan(plan, stream);
}

sten_status sten_batch_destroy(sten_batch_handle plan) {
    delete plan;
    return STEN_OK;
}

sten_status sten_batch_set_modes(sten_batch_handle plan, int32_t use_reg, hipStream_t stream) {
    if (plan == nullptr || (use_reg != 0 && use_reg != 1)) return STEN_ERR_ARG;
    const sten::Config saved = plan->cfg;
    plan->cfg.use_reg = use_reg;
    sten_status st = sten::finalize_plan(plan, stream);
    if (st != STEN_OK) {
        plan->cfg = saved;
        (void)sten::finalize_plan(plan, stream);
    }
    return st;
}

sten_status sten_batch_plan_info(sten_batch_handle plan, int32_t* info, int32_t n) {
    if (plan == nullptr || info == nullptr || n < 7) return STEN_ERR_ARG;
    info[0] = plan->cfg.block;
    info[1] = plan->cfg.lds_bytes;
    info[2] = plan->cfg.wg_per_cu;
    info[3] = plan->grid;
    info[4] = plan->n_lds;
    info[5] = plan->n_global;
    info[6] = plan->n_copy;
    if (n >= 9) {
        info[7] = plan->n_reg;
        info[8] = plan->cfg.use_reg;
    }
    return STEN_OK;
}

sten_status sten_batch_configure(sten_batch_handle plan, int32_t block, int32_t lds_bytes, int32_t wg_per_cu,
                                 hipStream_t stream) {
    using namespace sten;
    if (plan == nullptr) return STEN_ERR_ARG;
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024) return STEN_ERR_ARG;
    if (lds_bytes < 1024 || wg_per_cu < 1 || wg_per_cu > 32) return STEN_ERR_ARG;
    Config c;
    c.block = block;
    c.lds_bytes = lds_bytes;
    c.wg_per_cu = wg_per_cu;
    c.use_reg = plan->cfg.use_reg;
    const Config saved = plan->cfg;
    plan->cfg = c;
    sten_status st = finalize_plan(plan, stream);
    if (st != STEN_OK) {
        plan->cfg = saved;
        (void)finalize_plan(plan, stream);
    }
    return st;
}

sten_status sten_batch_autotune(sten_batch_handle plan, const char* tune_cache_path, int32_t reps, float* best_us,
                                hipStream_t stream) {
    using namespace sten;
    if (plan == nullptr || reps < 1) return STEN_ERR_ARG;
    const int limit = device_lds_limit();
    std::vector<Config> cands;
    for (int use_reg : {1, 0}) {
        for (int block : {256, 512, 1024}) {
            for (int kb : {32, 64, 80, 160}) {
                if (kb * 1024 > limit) continue;
                Config c;
                c.block = block;
                c.lds_bytes = kb * 1024;
                c.wg_per_cu = std::max(1, std::min(limit / (kb * 1024), 2048 / block));
                c.use_reg = use_reg;
                cands.push_back(c);
            }
        }
    }
    hipEvent_t e0, e1;
    hipError_t he = hipEventCreate(&e0);
    if (he != hipSuccess) return hip_fail(he);
    he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he);
    }
    const Config saved = plan->cfg;
    Config best = saved;
    float best_t = 1e30f;
    sten_status st = STEN_OK;
    for (const Config& cand : cands) {
        plan->cfg = cand;
        st = finalize_plan(plan, stream);
        if (st == STEN_ERR_PTR) {  // sends a grid without `work` to global mode: not a candidate
            st = STEN_OK;
            continue;
        }
        if (st != STEN_OK) break;
        if ((st = launch_plan(plan, stream)) != STEN_OK) break;  // warm-up
        if ((he = hipEventRecord(e0, stream)) != hipSuccess) { st = hip_fail(he); break; }
        for (int r = 0; r < reps && st == STEN_OK; ++r) st = launch_plan(plan, stream);
        if (st != STEN_OK) break;
        if ((he = hipEventRecord(e1, stream)) != hipSuccess) { st = hip_fail(he); break; }
        if ((he = hipEventSynchronize(e1)) != hipSuccess) { st = hip_fail(he); break; }
        float ms = 0.0f;
        if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { st = hip_fail(he); break; }
        const float us = ms * 1000.0f / reps;
        if (us < best_t) {
            best_t = us;
            best = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->cfg = (st == STEN_OK) ? best : saved;
    sten_status st2 = finalize_plan(plan, stream);
    if (st != STEN_OK) return st;
    if (st2 != STEN_OK) return st2;
    if (best_us != nullptr) *best_us = best_t;
    if (tune_cache_path != nullptr &&
        !cache_store(tune_cache_path, batch_key(plan->h_insts.data(), plan->count, plan->T), best, best_t))
        return STEN_ERR_ARG;
    return STEN_OK;
}

}  // extern "C"
