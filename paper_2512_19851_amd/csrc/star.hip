// General constant-coefficient star stencils of radius R (1..4) with up to
// four fused outputs: the generated-kernel side of the paper's frontend
// (Section III-C, code generation) for the class of slice expressions
//     out[R:-R, R:-R] = c0*A + cN1*A[up 1] + cS1*A[down 1] + cW1*A[left 1] + cE1*A[right 1]
//                            + ... + cER*A[right R]
// evaluated left to right (each product rounded, then added; no fused
// multiply-add). Ghost depth = R, the largest offset read (Section III-C).
// Node fusion (Section III-B): assignments with the same output shape and no
// dependence between them that read the same array run as one kernel, which
// reads the array once and writes every output.
//
// Kernel: a 256-lane workgroup stages a (16 + 2R) x (256 + 2R) block of the
// input in LDS (coalesced row loads; halo from L2), then each lane walks one
// column of 16 output rows, reading its 4R+1 neighbours from LDS once and
// feeding them to every fused output.
#include <algorithm>

#include "common.hpp"

namespace sten {
namespace {

constexpr int kStarBlock = 256;
constexpr int kStarRows = 16;

struct StarArgs {
    double c[4][17];  // per output: c0, then for k = 1..4: cn, cs, cw, ce
    double* out[4];
};

template <int R, int NOUT>
__global__ __launch_bounds__(kStarBlock) void star_kernel(const double* __restrict__ in, StarArgs a, int H, int W,
                                                          int64_t ld, uint32_t tiles_x) {
    constexpr int LW = kStarBlock + 2 * R;
    constexpr int LH = kStarRows + 2 * R;
    __shared__ double tile[LH * LW];
    const uint32_t t = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t ty = t / tiles_x;
    const uint32_t tx = t - ty * tiles_x;
    const int j0 = (int)tx * kStarBlock;  // first output column of the tile
    const int i0 = (int)ty * kStarRows;   // first output row of the tile
    for (int idx = threadIdx.x; idx < LH * LW; idx += kStarBlock) {
        const int r = idx / LW;
        const int cc = idx - r * LW;
        const int i = i0 - R + r;
        const int j = j0 - R + cc;
        tile[idx] = (i >= 0 && i < H && j >= 0 && j < W) ? in[(int64_t)i * ld + j] : 0.0;
    }
    __syncthreads();
    const int j = j0 + (int)threadIdx.x;
    if (j < R || j > W - 1 - R) return;
    const int lc = (int)threadIdx.x + R;
    for (int r = 0; r < kStarRows; ++r) {
        const int i = i0 + r;
        if (i < R || i > H - 1 - R) continue;
        const double* p = tile + (r + R) * LW + lc;
        const double ctr = p[0];
        double nb[R][4];
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            nb[k - 1][0] = p[-k * LW];
            nb[k - 1][1] = p[k * LW];
            nb[k - 1][2] = p[-k];
            nb[k - 1][3] = p[k];
        }
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
            double acc = a.c[o][0] * ctr;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
#pragma unroll
                for (int d = 0; d < 4; ++d) acc = acc + a.c[o][1 + 4 * (k - 1) + d] * nb[k - 1][d];
            }
            a.out[o][(int64_t)i * ld + j] = acc;
        }
    }
}

__global__ void star_copy_kernel(const double* __restrict__ src, double* __restrict__ d1, double* __restrict__ d2,
                                 int H, int W, int64_t ld) {
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / W;
        const int64_t j = idx - i * W;
        const double v = src[i * ld + j];
        d1[i * ld + j] = v;
        if (d2 != nullptr) d2[i * ld + j] = v;
    }
}

template <int R>
void launch_star_r(const double* in, const StarArgs& a, int nout, int H, int W, int64_t ld, hipStream_t s) {
    const uint32_t tiles_x = ceil_div(W, kStarBlock);
    const uint32_t tiles_y = ceil_div(H, kStarRows);
    const uint32_t grid = tiles_x * tiles_y;
    switch (nout) {
        case 1: star_kernel<R, 1><<<grid, kStarBlock, 0, s>>>(in, a, H, W, ld, tiles_x); break;
        case 2: star_kernel<R, 2><<<grid, kStarBlock, 0, s>>>(in, a, H, W, ld, tiles_x); break;
        case 3: star_kernel<R, 3><<<grid, kStarBlock, 0, s>>>(in, a, H, W, ld, tiles_x); break;
        default: star_kernel<R, 4><<<grid, kStarBlock, 0, s>>>(in, a, H, W, ld, tiles_x); break;
    }
}

void launch_star(const double* in, const StarArgs& a, int R, int nout, int H, int W, int64_t ld, hipStream_t s) {
    switch (R) {
        case 1: launch_star_r<1>(in, a, nout, H, W, ld, s); break;
        case 2: launch_star_r<2>(in, a, nout, H, W, ld, s); break;
        case 3: launch_star_r<3>(in, a, nout, H, W, ld, s); break;
        default: launch_star_r<4>(in, a, nout, H, W, ld, s); break;
    }
}

void fill_coef(const sten_star_coef& s, double* c) {
    c[0] = s.c0;
    for (int k = 0; k < 4; ++k) {
        c[1 + 4 * k + 0] = s.cn[k];
        c[1 + 4 * k + 1] = s.cs[k];
        c[1 + 4 * k + 2] = s.cw[k];
        c[1 + 4 * k + 3] = s.ce[k];
    }
}

sten_status check_star_dims(int64_t H, int64_t W, int64_t ld) {
    if (H < 0 || W < 0) return STEN_ERR_ARG;
    if (H > 0 && ld < W) return STEN_ERR_ARG;
    if (H > INT32_MAX / 2 || W > INT32_MAX / 2) return STEN_ERR_ARG;
    return STEN_OK;
}

}  // namespace
}  // namespace sten

extern "C" {

sten_status sten_star_f64(const double* in, double* const* outs, const sten_star_coef* coefs, int32_t nout, int64_t H,
                          int64_t W, int64_t ld, hipStream_t stream) {
    using namespace sten;
    if (nout < 1 || nout > 4 || coefs == nullptr || outs == nullptr) return STEN_ERR_ARG;
    const int R = coefs[0].radius;
    if (R < 1 || R > 4) return STEN_ERR_ARG;
    for (int o = 1; o < nout; ++o)
        if (coefs[o].radius != R) return STEN_ERR_ARG;  // fused outputs share the output shape
    sten_status st = check_star_dims(H, W, ld);
    if (st != STEN_OK || H == 0 || W == 0) return st;
    if (in == nullptr) return STEN_ERR_PTR;
    const size_t nb = span_bytes(H, W, ld, 8);
    for (int o = 0; o < nout; ++o) {
        if (outs[o] == nullptr) return STEN_ERR_PTR;
        if (overlaps(in, nb, outs[o], nb)) return STEN_ERR_ALIAS;
        for (int q = 0; q < o; ++q)
            if (overlaps(outs[q], nb, outs[o], nb)) return STEN_ERR_ALIAS;
    }
    if (!is_device_ptr(in)) return STEN_ERR_PTR;
    for (int o = 0; o < nout; ++o)
        if (!is_device_ptr(outs[o])) return STEN_ERR_PTR;
    if (H < 2 * R + 1 || W < 2 * R + 1) return STEN_OK;  // nothing to update
    StarArgs a{};
    for (int o = 0; o < nout; ++o) {
        fill_coef(coefs[o], a.c[o]);
        a.out[o] = outs[o];
    }
    launch_star(in, a, R, nout, (int)H, (int)W, ld, stream);
    return check_launch();
}

sten_status sten_star_iterate_f64(const double* u0, double* out, double* work, const sten_star_coef* coef,
                                  int64_t H, int64_t W, int64_t ld, int32_t T, hipStream_t stream) {
    using namespace sten;
    if (coef == nullptr || coef->radius < 1 || coef->radius > 4 || T < 0) return STEN_ERR_ARG;
    const int R = coef->radius;
    const bool active = H >= 2 * R + 1 && W >= 2 * R + 1 && T > 0;
    sten_status st = check_grid_args(u0, out, work, active && T >= 2, H, W, ld, T, 8);
    if (st != STEN_OK || H == 0 || W == 0) return st;
    const int h = (int)H, w = (int)W;
    const uint32_t blocks = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((H * W + 255) / 256, 65536));
    star_copy_kernel<<<blocks, 256, 0, stream>>>(u0, out, (active && T >= 2) ? work : nullptr, h, w, ld);
    if (!active) return check_launch();
    StarArgs a{};
    fill_coef(*coef, a.c[0]);
    const double* src = u0;
    for (int32_t k = 1; k <= T; ++k) {
        double* dst = ((T - k) % 2 == 0) ? out : work;
        a.out[0] = dst;
        launch_star(src, a, R, 1, h, w, ld, stream);
        src = dst;
    }
    return check_launch();
}

}  // extern "C"
