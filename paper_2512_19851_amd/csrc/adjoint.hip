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
// lambda_k = dL/du_k, which needs the forward states u_k: fused kernels of one
// or two transposed steps produce lambda_k from lambda_{k+1} and add each
// step's dot product, accumulated in FP64, into per-workgroup partial sums
// (each workgroup owns a fixed tile, so the sum is deterministic); a
// single-block kernel reduces the partials in a fixed order. Without dL/dc,
// a streaming kernel applies several transposed steps per launch.
//
// FP32 arithmetic, neighbour terms in the order N, S, W, E (missing or ring
// neighbours contribute an exact zero), then one multiplication by c and, on
// the ring, one addition of the point's own value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "common.hpp"
#include "stream_common.hpp"

namespace sten {

// Forward FP32 sweep launcher exported by sweep.hip.
void launch_sweep_f32_internal(const float* in, float* out, int H, int W, int64_t ld, float c, hipStream_t s);

namespace {

constexpr int kAdjBlock = 256;
constexpr int kAdjRows = 2;       // rows per tile of the fused one-step kernel

constexpr int kAdjTileBlock = kWave;  // one wave (256 columns) per workgroup of the fused one-step kernel

// Sum of a double over a workgroup of NT lanes (fixed order: lanes by shuffle tree, then waves in order).
template <int NT>
__device__ double block_sum(double v) {
    __shared__ double wsum[NT / kWave];
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    if (lane == 0) wsum[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / kWave; ++w) t += wsum[w];
    __syncthreads();
    return t;
}

// Both kernels below evaluate one transposed step per point exactly as the
// definition above: the four neighbour terms in the order N, S, W, E, each an
// exact zero unless that neighbour is an interior point, summed left to right
// in FP32, one multiplication by c, and on the ring one addition of the
// point's own value first (g + c * sum). Every grid point is written.
//
// Column facts of one element: column j of a W-column grid.
struct AdjCol {
    bool in;    // j is an interior column
    bool west;  // j - 1 is an interior column
    bool east;  // j + 1 is an interior column
};
__device__ __forceinline__ AdjCol adj_col(int j, int W) {
    return AdjCol{j >= 1 && j <= W - 2, j >= 2 && j <= W - 1, j >= 0 && j <= W - 3};
}
__device__ __forceinline__ bool adj_interior_row(int r, int H) { return r >= 1 && r <= H - 2; }

// One transposed point: n, s, w, e are the four neighbours' values, m the
// point's own; rn, rs: rows above and below are interior; rin: own row interior.
__device__ __forceinline__ float adj_point(float n, float s, float w, float e, float m, bool rn, bool rs, bool rin,
                                           const AdjCol& col, float c) {
    float t = (rn && col.in ? n : 0.0f) + (rs && col.in ? s : 0.0f);
    t = t + (rin && col.west ? w : 0.0f);
    t = t + (rin && col.east ? e : 0.0f);
    const float v = c * t;
    return (rin && col.in) ? v : m + v;
}

constexpr int kAdjV = 4;  // floats per lane: one 16-byte vector

// Row r of g (zeros outside the grid) into x: columns j0 .. j0+3.
template <bool VEC>
__device__ __forceinline__ void adj_load(const float* __restrict__ g, int r, int H, int W, int64_t ld, int j0,
                                         float (&x)[kAdjV]) {
    if (r < 0 || r >= H) {
#pragma unroll
        for (int e = 0; e < kAdjV; ++e) x[e] = 0.0f;
        return;
    }
    const float* row = g + (int64_t)r * ld;
    if (VEC && j0 >= 0 && j0 + kAdjV <= W) {
        typedef float F4 __attribute__((ext_vector_type(4)));
        const F4 v = *reinterpret_cast<const F4*>(row + j0);
#pragma unroll
        for (int e = 0; e < kAdjV; ++e) x[e] = v[e];
    } else {
#pragma unroll
        for (int e = 0; e < kAdjV; ++e) x[e] = (j0 + e >= 0 && j0 + e < W) ? row[j0 + e] : 0.0f;
    }
}

// Columns j0 .. j0+3 of row r (inside the grid) where they lie in [lo, hi).
template <bool VEC>
__device__ __forceinline__ void adj_store(float* __restrict__ out, int r, int64_t ld, int j0, int lo, int hi,
                                          const float (&x)[kAdjV]) {
    float* row = out + (int64_t)r * ld;
    if (VEC && j0 >= lo && j0 + kAdjV <= hi) {
        typedef float F4 __attribute__((ext_vector_type(4)));
        F4 v;
#pragma unroll
        for (int e = 0; e < kAdjV; ++e) v[e] = x[e];
        *reinterpret_cast<F4*>(row + j0) = v;
    } else {
#pragma unroll
        for (int e = 0; e < kAdjV; ++e)
            if (j0 + e >= lo && j0 + e < hi) row[j0 + e] = x[e];
    }
}

// One transposed step, fused with the dL/dc term when u is given:
// partials[block] (+)= sum over this tile's interior points m of
// g[m] * nbrsum(u)[m] (FP32 neighbour sum in the order N, S, W, E, product
// and sum in FP64). A workgroup of one wave owns a tile of ROWS rows by 256
// columns (4 floats per lane; small tiles, so that even a 1024^2 grid has
// thousands of waves); a lane keeps its column vector of the tile's ROWS + 2
// rows of g (and u) in registers and walks down; the neighbours across lanes come from DPP lane
// shifts, and the wave's two edge lanes load the one column that lies in the
// next tile. Each workgroup owns a fixed tile, so the partial sums, and their
// reduction, are deterministic.
template <int ROWS, bool VEC, bool DOT>
__global__ __launch_bounds__(kAdjTileBlock) void adjoint_tile_kernel(const float* __restrict__ g,
                                                                 const float* __restrict__ u,
                                                                 float* __restrict__ out,
                                                                 double* __restrict__ partials, int accumulate,
                                                                 int H, int W, int64_t ld, float c,
                                                                 uint32_t tiles_x) {
    using stream::lane_from_lower;
    using stream::lane_from_upper;
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t ty = tile / tiles_x;
    const uint32_t tx = tile - ty * tiles_x;
    const int lane = threadIdx.x & (kWave - 1);
    const int j0 = ((int)tx * kAdjTileBlock + (int)threadIdx.x) * kAdjV;
    const int i0 = (int)ty * ROWS;  // first output row (every grid row is an output row)
    float a[ROWS + 2][kAdjV];
    float q[DOT ? ROWS + 2 : 1][kAdjV];
#pragma unroll
    for (int k = 0; k < ROWS + 2; ++k) {
        adj_load<VEC>(g, i0 - 1 + k, H, W, ld, j0, a[k]);
        if constexpr (DOT) adj_load<VEC>(u, i0 - 1 + k, H, W, ld, j0, q[k]);
    }
    AdjCol col[kAdjV];
#pragma unroll
    for (int e = 0; e < kAdjV; ++e) col[e] = adj_col(j0 + e, W);
    const bool edge_w = lane == 0 && j0 > 0 && j0 <= W;                  // column j0 - 1 lies in another wave
    const bool edge_e = lane == kWave - 1 && j0 + kAdjV < W;             // column j0 + 4 lies in another wave
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int r = i0 + k;
        if (r < H) {  // uniform over the workgroup
            const float* grow = g + (int64_t)r * ld;
            float lft = lane_from_lower(a[k + 1][kAdjV - 1]);
            float rgt = lane_from_upper(a[k + 1][0]);
            if (edge_w) lft = grow[j0 - 1];
            if (edge_e) rgt = grow[j0 + kAdjV];
            const bool rn = adj_interior_row(r - 1, H), rs = adj_interior_row(r + 1, H), rin = adj_interior_row(r, H);
            float o[kAdjV];
#pragma unroll
            for (int e = 0; e < kAdjV; ++e) {
                const float w = e == 0 ? lft : a[k + 1][e > 0 ? e - 1 : 0];
                const float ea = e == kAdjV - 1 ? rgt : a[k + 1][e < kAdjV - 1 ? e + 1 : 0];
                o[e] = adj_point(a[k][e], a[k + 2][e], w, ea, a[k + 1][e], rn, rs, rin, col[e], c);
            }
            adj_store<VEC>(out, r, ld, j0, 0, W, o);
            if constexpr (DOT) {
                if (rin) {
                    const float* urow = u + (int64_t)r * ld;
                    float ul = lane_from_lower(q[k + 1][kAdjV - 1]);
                    float ur = lane_from_upper(q[k + 1][0]);
                    if (edge_w) ul = urow[j0 - 1];
                    if (edge_e) ur = urow[j0 + kAdjV];
#pragma unroll
                    for (int e = 0; e < kAdjV; ++e) {
                        if (col[e].in) {
                            const float uw = e == 0 ? ul : q[k + 1][e > 0 ? e - 1 : 0];
                            const float ue = e == kAdjV - 1 ? ur : q[k + 1][e < kAdjV - 1 ? e + 1 : 0];
                            float ns = q[k][e] + q[k + 2][e];
                            ns = ns + uw;
                            ns = ns + ue;
                            acc += (double)a[k + 1][e] * (double)ns;
                        }
                    }
                }
            }
        }
    }
    if constexpr (DOT) {
        const double t = block_sum<kAdjTileBlock>(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = accumulate ? partials[blockIdx.x] + t : t;
    }
}

// The transposed step at one point (r, j) read straight from g (zeros outside
// the grid): the value a wave's edge lane needs one column past its tile.
__device__ __forceinline__ float adj_point_at(const float* __restrict__ g, int r, int j, int H, int W, int64_t ld,
                                              float c) {
    auto at = [&](int rr, int jj) -> float {
        return (rr >= 0 && rr < H && jj >= 0 && jj < W) ? g[(int64_t)rr * ld + jj] : 0.0f;
    };
    return adj_point(at(r - 1, j), at(r + 1, j), at(r, j - 1), at(r, j + 1), at(r, j), adj_interior_row(r - 1, H),
                     adj_interior_row(r + 1, H), adj_interior_row(r, H), adj_col(j, W), c);
}

// The dL/dc term of one tile row: sum over the row's interior points m of g[m] * nbrsum(u)[m], the
// neighbour sum in FP32 in the order N, S, W, E, product and sum in FP64, elements in order.
template <bool VEC>
__device__ __forceinline__ void adj_dot_row(double& acc, const float (&gm)[kAdjV], const float (&un)[kAdjV],
                                            const float (&um)[kAdjV], const float (&us)[kAdjV],
                                            const float* __restrict__ urow, int j0, bool edge_w, bool edge_e,
                                            const AdjCol (&col)[kAdjV]) {
    float ul = stream::lane_from_lower(um[kAdjV - 1]);
    float ur = stream::lane_from_upper(um[0]);
    if (edge_w) ul = urow[j0 - 1];
    if (edge_e) ur = urow[j0 + kAdjV];
#pragma unroll
    for (int e = 0; e < kAdjV; ++e) {
        if (col[e].in) {
            const float uw = e == 0 ? ul : um[e > 0 ? e - 1 : 0];
            const float ue = e == kAdjV - 1 ? ur : um[e < kAdjV - 1 ? e + 1 : 0];
            float ns = un[e] + us[e];
            ns = ns + uw;
            ns = ns + ue;
            acc += (double)gm[e] * (double)ns;
        }
    }
}

// Two transposed steps with their dL/dc terms in one launch, on the tiles of
// the one-step kernel (2 rows by 256 columns per one-wave workgroup):
// lambda_k = S^T lambda_{k+1} on the tile's rows and one row either side
// (from 6 loaded rows of lambda_{k+1}; the wave's edge lanes compute the one
// column past the tile from g directly), then lambda_{k-1} = S^T lambda_k on
// the tile's rows. Every value is the one-step kernel's, and each step's sum is
// reduced over the workgroup and added to the partial sum in the order two
// one-step launches would add them, so the results are bit-identical to two
// launches of the one-step kernel.
template <bool VEC>
__global__ __launch_bounds__(kAdjTileBlock) void adjoint_tile2_kernel(
    const float* __restrict__ g, const float* __restrict__ u1, const float* __restrict__ u2,
    float* __restrict__ out, double* __restrict__ partials, int accumulate, int H, int W, int64_t ld, float c,
    uint32_t tiles_x) {
    constexpr int R = kAdjRows;  // 2
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t ty = tile / tiles_x;
    const uint32_t tx = tile - ty * tiles_x;
    const int lane = threadIdx.x & (kWave - 1);
    const int j0 = ((int)tx * kAdjTileBlock + (int)threadIdx.x) * kAdjV;
    const int i0 = (int)ty * R;
    const bool edge_w = lane == 0 && j0 > 0 && j0 <= W;
    const bool edge_e = lane == kWave - 1 && j0 + kAdjV < W;
    AdjCol col[kAdjV];
#pragma unroll
    for (int e = 0; e < kAdjV; ++e) col[e] = adj_col(j0 + e, W);

    float a[R + 4][kAdjV];   // lambda_{k+1}, rows i0-2 .. i0+R+1
    float q1[R + 2][kAdjV];  // u_k, rows i0-1 .. i0+R
    float q2[R + 2][kAdjV];  // u_{k-1}, rows i0-1 .. i0+R
#pragma unroll
    for (int m = 0; m < R + 4; ++m) adj_load<VEC>(g, i0 - 2 + m, H, W, ld, j0, a[m]);
#pragma unroll
    for (int m = 0; m < R + 2; ++m) {
        adj_load<VEC>(u1, i0 - 1 + m, H, W, ld, j0, q1[m]);
        adj_load<VEC>(u2, i0 - 1 + m, H, W, ld, j0, q2[m]);
    }

    // step 1: lambda_k on rows i0-1 .. i0+R (zeros outside the grid, as a one-step launch's loads give)
    float b[R + 2][kAdjV];
    double acc1 = 0.0;
#pragma unroll
    for (int m = 0; m < R + 2; ++m) {
        const int r = i0 - 1 + m;
        if (r < 0 || r >= H) {
#pragma unroll
            for (int e = 0; e < kAdjV; ++e) b[m][e] = 0.0f;
            continue;
        }
        const float* grow = g + (int64_t)r * ld;
        float lft = stream::lane_from_lower(a[m + 1][kAdjV - 1]);
        float rgt = stream::lane_from_upper(a[m + 1][0]);
        if (edge_w) lft = grow[j0 - 1];
        if (edge_e) rgt = grow[j0 + kAdjV];
        const bool rn = adj_interior_row(r - 1, H), rs = adj_interior_row(r + 1, H), rin = adj_interior_row(r, H);
#pragma unroll
        for (int e = 0; e < kAdjV; ++e) {
            const float w = e == 0 ? lft : a[m + 1][e > 0 ? e - 1 : 0];
            const float ea = e == kAdjV - 1 ? rgt : a[m + 1][e < kAdjV - 1 ? e + 1 : 0];
            b[m][e] = adj_point(a[m][e], a[m + 2][e], w, ea, a[m + 1][e], rn, rs, rin, col[e], c);
        }
        // the tile's own rows: the step's dL/dc term, as the one-step kernel sums it
        if (m >= 1 && m <= R && rin)
            adj_dot_row<VEC>(acc1, a[m + 1], q1[m - 1], q1[m], q1[m + 1], u1 + (int64_t)r * ld, j0, edge_w, edge_e,
                             col);
    }
    // step 2: lambda_{k-1} on the tile's rows; the edge lanes' neighbour column of lambda_k from g
    double acc2 = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = i0 + k;
        if (r >= H) continue;  // uniform over the workgroup
        float lft = stream::lane_from_lower(b[k + 1][kAdjV - 1]);
        float rgt = stream::lane_from_upper(b[k + 1][0]);
        if (edge_w) lft = adj_point_at(g, r, j0 - 1, H, W, ld, c);
        if (edge_e) rgt = adj_point_at(g, r, j0 + kAdjV, H, W, ld, c);
        const bool rn = adj_interior_row(r - 1, H), rs = adj_interior_row(r + 1, H), rin = adj_interior_row(r, H);
        float o[kAdjV];
#pragma unroll
        for (int e = 0; e < kAdjV; ++e) {
            const float w = e == 0 ? lft : b[k + 1][e > 0 ? e - 1 : 0];
            const float ea = e == kAdjV - 1 ? rgt : b[k + 1][e < kAdjV - 1 ? e + 1 : 0];
            o[e] = adj_point(b[k][e], b[k + 2][e], w, ea, b[k + 1][e], rn, rs, rin, col[e], c);
        }
        adj_store<VEC>(out, r, ld, j0, 0, W, o);
        if (rin) adj_dot_row<VEC>(acc2, b[k + 1], q2[k], q2[k + 1], q2[k + 2], u2 + (int64_t)r * ld, j0, edge_w, edge_e, col);
    }
    const double t1 = block_sum<kAdjTileBlock>(acc1);
    const double t2 = block_sum<kAdjTileBlock>(acc2);
    if (threadIdx.x == 0) {
        const double p1 = accumulate ? partials[blockIdx.x] + t1 : t1;
        partials[blockIdx.x] = p1 + t2;
    }
}

// Several transposed steps per launch (no dL/dc): the streaming form of
// temporal blocking, as in the forward kernel. One wave owns a strip of 256
// loaded columns (4 floats per lane) and a band of output rows, and walks the
// band once: each step loads one row (level 0) and, for s = 1..TL, computes
// level s of the row s behind the loaded one from the two level-(s-1) rows it
// keeps and the level-(s-1) row just produced; level TL of the row TL behind
// is stored. Bands cover every row and strips every column, ring included,
// since the transposed step writes every point. A level's row r is computed
// from rows a (r - dir, kept from the step before) and b (r + dir), so a + b
// is N + S or S + N: the same bits, IEEE addition being commutative (a
// missing term is an exact zero either way).
//
// Rows and columns outside the grid are loaded clamped to the grid, and the
// strip's halo columns see a zero past the wave's edge lanes: none of these
// points is interior, so the masked expression never lets their values reach
// a point (and plain groups, see below, never hold such points next to a
// stored one: the halo is at least TL columns wide, and the rows a plain group
// computes all lie in [2, H-3]). In a group whose level rows all lie in
// [2, H-3], on a strip whose loaded columns all lie in [2, W-3], every point
// and its four neighbours are interior, so the plain five-point expression is
// the transposed step there; elsewhere every term is masked.
constexpr int kAdjStreamA = 4;       // rows loaded ahead
constexpr int kAdjStreamLevels = 8;  // transposed steps per launch at most

// Tuning setting (read once per call; every accepted value gives the same bits):
// transposed steps per launch, 0 for the built-in choice.
std::atomic<int> g_adj_levels{0};

template <int A>
struct AdjRing {
    static constexpr int P = A + 2;
    static constexpr int U = (P % 3 == 0) ? P : 3 * P;  // steps per group: whole periods of every rotation
};

// One level of the row r = (loaded row) - dir*s: a = row r - dir, m = row r, b = row r + dir.
template <bool MASK>
__device__ __forceinline__ void adj_stream_level(const float (&a)[kAdjV], const float (&m)[kAdjV],
                                                 const float (&b)[kAdjV], float (&res)[kAdjV], float c, int r,
                                                 int dir, int H, const AdjCol (&col)[kAdjV]) {
    const float lft = stream::lane_from_lower(m[kAdjV - 1]);  // column j0 - 1
    const float rgt = stream::lane_from_upper(m[0]);          // column j0 + 4
    if constexpr (!MASK) {
#pragma unroll
        for (int e = 0; e < kAdjV; ++e) {
            const float w = e == 0 ? lft : m[e > 0 ? e - 1 : 0];
            const float ea = e == kAdjV - 1 ? rgt : m[e < kAdjV - 1 ? e + 1 : 0];
            float t = a[e] + b[e];
            t = t + w;
            t = t + ea;
            res[e] = c * t;
        }
    } else {
        const bool ia = adj_interior_row(r - dir, H), ib = adj_interior_row(r + dir, H), rin = adj_interior_row(r, H);
#pragma unroll
        for (int e = 0; e < kAdjV; ++e) {
            const float w = e == 0 ? lft : m[e > 0 ? e - 1 : 0];
            const float ea = e == kAdjV - 1 ? rgt : m[e < kAdjV - 1 ? e + 1 : 0];
            res[e] = adj_point(a[e], b[e], w, ea, m[e], ia, ib, rin, col[e], c);
        }
    }
}

// One step: the level-0 row L (x) enters; levels 1..NACT advance by one row each.
template <int TL, int NACT, bool MASK>
__device__ __forceinline__ void adj_stream_step(float (&w0)[TL][kAdjV], float (&w1)[TL][kAdjV],
                                                const float (&a0)[kAdjV], const float (&b0)[kAdjV],
                                                const float (&x)[kAdjV], float (&top)[kAdjV], int L, int dir, int H,
                                                float c, const AdjCol (&col)[kAdjV]) {
    if constexpr (NACT >= 1) {
        float cur[kAdjV];
        adj_stream_level<MASK>(a0, b0, x, cur, c, L - dir, dir, H, col);
#pragma unroll
        for (int s = 2; s <= NACT; ++s) {
            float nv[kAdjV];
            adj_stream_level<MASK>(w0[s - 1], w1[s - 1], cur, nv, c, L - dir * s, dir, H, col);
#pragma unroll
            for (int e = 0; e < kAdjV; ++e) {
                w0[s - 1][e] = w1[s - 1][e];
                w1[s - 1][e] = cur[e];
                cur[e] = nv[e];
            }
        }
        if constexpr (NACT < TL) {
#pragma unroll
            for (int e = 0; e < kAdjV; ++e) {
                w0[NACT][e] = w1[NACT][e];
                w1[NACT][e] = cur[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < kAdjV; ++e) top[e] = cur[e];
        }
    }
}

// Steps 0 .. 2*TL-1: level s is complete from step 2s on. `plain`: every row these steps compute
// lies in [2, H-3] on a strip of interior columns.
template <int TL, int A, int K, int EDGE>
__device__ __forceinline__ void adj_stream_prologue(float (&w0)[TL][kAdjV], float (&w1)[TL][kAdjV],
                                                    float (&ring)[AdjRing<A>::P][kAdjV], const float* __restrict__ g,
                                                    int L0, int dir, int H, int W, int64_t ld, int j0, float c,
                                                    const AdjCol (&col)[kAdjV], bool plain) {
    constexpr int P = AdjRing<A>::P;
    if constexpr (K < 2 * TL) {
        float unused[kAdjV];
        if (plain)
            adj_stream_step<TL, K / 2, false>(w0, w1, ring[(K + P - 2) % P], ring[(K + P - 1) % P], ring[K % P],
                                              unused, L0 + dir * K, dir, H, c, col);
        else
            adj_stream_step<TL, K / 2, true>(w0, w1, ring[(K + P - 2) % P], ring[(K + P - 1) % P], ring[K % P],
                                             unused, L0 + dir * K, dir, H, c, col);
        stream::stream_load<float, kAdjV, EDGE>(g, L0 + dir * (K + A), H, W, ld, j0, ring[(K + A) % P]);
        __builtin_amdgcn_sched_barrier(0);
        adj_stream_prologue<TL, A, K + 1, EDGE>(w0, w1, ring, g, L0, dir, H, W, ld, j0, c, col, plain);
    }
}

// One wave's band [rb, re) of a strip loading columns [cs, cs + 256) and storing [olo, ohi).
// EDGE 0: loaded columns all in [2, W-3], whole-vector loads and stores; EDGE 1: loaded columns
// inside the grid, whole-vector loads and stores, masked terms everywhere; EDGE 2: clamped loads,
// masked terms everywhere, stores column by column.
template <int TL, int A, int EDGE>
__device__ __forceinline__ void adj_stream_band(const float* __restrict__ g, float* __restrict__ out, int H, int W,
                                                int64_t ld, float c, int cs, int olo, int ohi, int rb, int re,
                                                int dir) {
    constexpr int P = AdjRing<A>::P;
    constexpr int U = AdjRing<A>::U;
    const int j0 = cs + (int)threadIdx.x * kAdjV;
    AdjCol col[kAdjV];
#pragma unroll
    for (int e = 0; e < kAdjV; ++e) col[e] = adj_col(j0 + e, W);
    const bool st_lane = (j0 >= olo) && (j0 + kAdjV <= ohi);
    const uint32_t voff_vec = st_lane ? (uint32_t)j0 * 4u : stream::kDropOffset;
    uint32_t voff_el[kAdjV];
#pragma unroll
    for (int e = 0; e < kAdjV; ++e)
        voff_el[e] = (j0 + e >= olo && j0 + e < ohi) ? (uint32_t)(j0 + e) * 4u : stream::kDropOffset;

    const int L0 = dir > 0 ? rb - TL : re - 1 + TL;
    const int nsteps = (re - rb) + 2 * TL;
    float w0[TL][kAdjV], w1[TL][kAdjV];
    float ring[P][kAdjV];
#pragma unroll
    for (int i = 0; i < A; ++i) stream::stream_load<float, kAdjV, EDGE>(g, L0 + dir * i, H, W, ld, j0, ring[i]);
    {
        // the prologue's level rows lie in [min(L0, Le) - TL, max(L0, Le) + TL], Le its last loaded row
        const int Le = L0 + dir * (2 * TL - 1);
        const bool plain = EDGE == 0 && min(L0, Le) - TL >= 2 && max(L0, Le) + TL <= H - 3;
        adj_stream_prologue<TL, A, 0, EDGE>(w0, w1, ring, g, L0, dir, H, W, ld, j0, c, col, plain);
    }

    const int ngroups = (nsteps - 2 * TL + U - 1) / U;
    for (int k = 0; k < ngroups; ++k) {
        const int gs = 2 * TL + k * U;
        const int La = L0 + dir * gs, Lb = L0 + dir * (gs + U - 1);
        // the level rows of this group lie in [min(La, Lb) - TL, max(La, Lb) + TL]
        const bool plain = EDGE == 0 && min(La, Lb) - TL >= 2 && max(La, Lb) + TL <= H - 3;
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int t = 2 * TL + i;  // step index modulo U
            const int L = L0 + dir * (gs + i);
            float top[kAdjV];
            if (plain)
                adj_stream_step<TL, TL, false>(w0, w1, ring[(t + P - 2) % P], ring[(t + P - 1) % P], ring[t % P], top,
                                               L, dir, H, c, col);
            else
                adj_stream_step<TL, TL, true>(w0, w1, ring[(t + P - 2) % P], ring[(t + P - 1) % P], ring[t % P], top,
                                              L, dir, H, c, col);
            stream::stream_load<float, kAdjV, EDGE>(g, L + dir * A, H, W, ld, j0, ring[(t + A) % P]);
            stream::stream_store<float, kAdjV, EDGE>(out, L - dir * TL, ld, W, gs + i < nsteps, voff_vec, voff_el,
                                                     top);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Strip layout. Flush (flush != 0: 16-byte aligned rows, W a multiple of 4 and at least 256):
// strip 0 loads columns [0, 256) and stores [0, 256 - HALO); strip k loads from k*OW and stores
// [k*OW + HALO, (k+1)*OW + HALO); the last strip loads the grid's last 256 columns and stores
// [W - 256 + HALO, W). Every load stays inside the grid, and the last strip's stores may overlap
// its neighbour's with the same bits. Otherwise strip k loads from k*OW - HALO and stores [k*OW,
// (k+1)*OW) within the grid. Band b covers rows [b*band, (b+1)*band) within the grid; even bands
// walk down, odd bands up.
// Occupancy: 4 waves per SIMD (128 VGPRs) up to 5 levels, 3 (168) above; uncapped, the masked path's
// registers would hold the 8-level kernel to 2 waves per SIMD.
template <int TL, int A>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(TL <= 5 ? 4 : 3))) void adjoint_stream_kernel(const float* __restrict__ g, float* __restrict__ out,
                                                               int H, int W, int64_t ld, float c, uint32_t strips,
                                                               int band, int flush) {
    constexpr int HALO = (TL + kAdjV - 1) / kAdjV * kAdjV;
    constexpr int OW = kWave * kAdjV - 2 * HALO;
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t bi = tile / strips;
    const uint32_t strip = tile - bi * strips;
    int cs, olo, ohi;
    if (flush) {
        const bool last = strip == strips - 1;
        cs = last ? W - kWave * kAdjV : (int)strip * OW;
        olo = strip == 0 ? 0 : cs + HALO;
        ohi = last ? W : cs + HALO + OW;
    } else {
        cs = (int)strip * OW - HALO;
        olo = max(cs + HALO, 0);
        ohi = min(cs + HALO + OW, W);
    }
    const int rb = (int)bi * band;
    const int re = min(rb + band, H);
    const int dir = (bi & 1) ? -1 : 1;
    if (flush && cs >= 2 && cs + kWave * kAdjV <= W - 2)
        adj_stream_band<TL, A, 0>(g, out, H, W, ld, c, cs, olo, ohi, rb, re, dir);
    else if (flush)
        adj_stream_band<TL, A, 1>(g, out, H, W, ld, c, cs, olo, ohi, rb, re, dir);
    else
        adj_stream_band<TL, A, 2>(g, out, H, W, ld, c, cs, olo, ohi, rb, re, dir);
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
    const double t = block_sum<kAdjBlock>(v);
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

inline uint32_t adj_tiles_x(int64_t W) { return ceil_div(W, (int64_t)kAdjTileBlock * kAdjV); }
inline uint32_t adj_blocks(int64_t H, int64_t W) { return adj_tiles_x(W) * ceil_div(H, kAdjRows); }

template <bool VEC>
void launch_adjoint_step(const float* g, const float* u, float* out, double* partials, int accumulate, int H, int W,
                         int64_t ld, float c, hipStream_t s) {
    const uint32_t nb = adj_blocks(H, W);
    if (u != nullptr && partials != nullptr)
        adjoint_tile_kernel<kAdjRows, VEC, true><<<nb, kAdjTileBlock, 0, s>>>(g, u, out, partials, accumulate, H,
                                                                             W, ld, c, adj_tiles_x(W));
    else
        adjoint_tile_kernel<kAdjRows, VEC, false><<<nb, kAdjTileBlock, 0, s>>>(g, nullptr, out, nullptr, 0, H, W, ld,
                                                                              c, adj_tiles_x(W));
}

// Waves of one kernel that fit on the device at once (one wave per workgroup).
int adj_resident_waves(const void* kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess)
        return 0;
    return cus * per_cu;
}

template <bool VEC>
void launch_adjoint_step2(const float* g, const float* u1, const float* u2, float* out, double* partials,
                          int accumulate, int H, int W, int64_t ld, float c, hipStream_t s) {
    adjoint_tile2_kernel<VEC><<<adj_blocks(H, W), kAdjTileBlock, 0, s>>>(g, u1, u2, out, partials, accumulate, H, W,
                                                                         ld, c, adj_tiles_x(W));
}

template <int TL>
void launch_adjoint_stream_levels(const float* g, float* out, int H, int W, int64_t ld, float c, bool vec,
                                  hipStream_t s) {
    constexpr int HALO = (TL + kAdjV - 1) / kAdjV * kAdjV;
    constexpr int OW = kWave * kAdjV - 2 * HALO;
    const bool flush = vec && W % kAdjV == 0 && W >= kWave * kAdjV;
    const uint32_t strips = flush ? ceil_div(W - kWave * kAdjV, OW) + 1 : ceil_div(W, OW);
    // the tallest bands that still give every resident wave slot a band, and at least 2*TL rows
    static const int waves =
        adj_resident_waves(reinterpret_cast<const void*>(&adjoint_stream_kernel<TL, kAdjStreamA>));
    const int64_t fit = std::max<int64_t>(1, (waves > 0 ? waves : 1024) / (int64_t)strips);
    const int band = (int)std::max<int64_t>(2 * TL, (H + fit - 1) / fit);
    const uint32_t bands = ceil_div(H, band);
    adjoint_stream_kernel<TL, kAdjStreamA><<<strips * bands, kWave, 0, s>>>(g, out, H, W, ld, c, strips, band,
                                                                             flush ? 1 : 0);
}

// One launch of `levels` transposed steps (1..kAdjStreamLevels) from g into out.
void launch_adjoint_stream(const float* g, float* out, int H, int W, int64_t ld, float c, int levels, bool vec,
                           hipStream_t s) {
    switch (levels) {
        case 1: launch_adjoint_stream_levels<1>(g, out, H, W, ld, c, vec, s); break;
        case 2: launch_adjoint_stream_levels<2>(g, out, H, W, ld, c, vec, s); break;
        case 3: launch_adjoint_stream_levels<3>(g, out, H, W, ld, c, vec, s); break;
        case 4: launch_adjoint_stream_levels<4>(g, out, H, W, ld, c, vec, s); break;
        case 5: launch_adjoint_stream_levels<5>(g, out, H, W, ld, c, vec, s); break;
        case 6: launch_adjoint_stream_levels<6>(g, out, H, W, ld, c, vec, s); break;
        case 7: launch_adjoint_stream_levels<7>(g, out, H, W, ld, c, vec, s); break;
        default: launch_adjoint_stream_levels<8>(g, out, H, W, ld, c, vec, s); break;  // levels == 8
    }
}

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
    const bool vec = ((((uintptr_t)lam_in | (uintptr_t)lam_out | (need_work ? (uintptr_t)work : 0) |
                        (states != nullptr ? (uintptr_t)states : 0)) % 16) == 0) && ld % kAdjV == 0;
    const float* src = lam_in;
    if (states != nullptr && partials != nullptr) {
        // fused launches of two steps (the last one alone when nsteps is odd): lambda from lambda, plus
        // each step's dL/dc term; the last launch writes lam_out
        const int launches = (nsteps + 1) / 2;
        int32_t s = 1;  // the next step: lambda_{k1 - s} from lambda_{k1 - s + 1}, with state u_{k1 - s}
        for (int l = 1; l <= launches; ++l) {
            float* dst = ((launches - l) % 2 == 0) ? lam_out : work;
            const float* u = states + (int64_t)(nsteps - s) * pstride;
            const int acc = (s == 1 && reset) ? 0 : 1;
            if (s + 1 <= nsteps) {
                const float* u_next = states + (int64_t)(nsteps - s - 1) * pstride;
                if (vec)
                    launch_adjoint_step2<true>(src, u, u_next, dst, partials, acc, h, w, ld, c, stream);
                else
                    launch_adjoint_step2<false>(src, u, u_next, dst, partials, acc, h, w, ld, c, stream);
                s += 2;
            } else {
                if (vec)
                    launch_adjoint_step<true>(src, u, dst, partials, acc, h, w, ld, c, stream);
                else
                    launch_adjoint_step<false>(src, u, dst, partials, acc, h, w, ld, c, stream);
                s += 1;
            }
            src = dst;
        }
        return check_launch();
    }
    // no dL/dc: several steps per launch, the steps split as evenly as the launch count allows; the
    // last launch writes lam_out
    // built-in: 3 steps per launch on grids of up to 2^23 points, where the 2*TL-row bands of deeper
    // launches leave most wave slots empty (us per step at 3 / 4 / 8 steps per launch: 1024^2 2.2 /
    // 3.0 / 3.7, 2048^2 3.2 / 4.0 / 4.5), and 8 above (4096^2: 6.7 at 8, 7.7 at 4, 10.0 at 3)
    const int tuned = g_adj_levels.load(std::memory_order_relaxed);
    const int per_launch = tuned > 0 ? tuned : (H * W <= ((int64_t)1 << 23) ? 3 : kAdjStreamLevels);
    const int launches = (nsteps + per_launch - 1) / per_launch;
    const int base = nsteps / launches, extra = nsteps % launches;
    for (int k = 1; k <= launches; ++k) {
        const int lev = base + (k <= extra ? 1 : 0);
        float* dst = ((launches - k) % 2 == 0) ? lam_out : work;
        launch_adjoint_stream(src, dst, h, w, ld, c, lev, vec, stream);
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

sten_status sten_tune_adjoint_levels(int32_t levels) {
    if (levels < 0 || levels > sten::kAdjStreamLevels) return STEN_ERR_ARG;
    sten::g_adj_levels.store(levels, std::memory_order_relaxed);
    return STEN_OK;
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
