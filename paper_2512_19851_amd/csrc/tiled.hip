// Tiled execution of the FP64 method on one GPU: the paper's chare layout and
// DAG-node execution (Section III-C, data layout and DAG execution), with all
// tiles on one device.
//
//  * The H x W grid is split into pr x pc tiles ("chares"). Each tile holds
//    its owned block plus a depth-1 ghost frame (the ghost depth of the
//    five-point stencil), in two buffers (the ping-pong pair), and one send
//    buffer per edge that has a neighbour.
//  * Before a sweep reads an array, its ghosts are refreshed if the array's
//    local generation epoch differs from its ghost epoch: on the
//    communication stream, after waiting for the compute event, a pack kernel
//    copies every tile's boundary strips into its send buffers and an unpack
//    kernel copies each neighbour's send buffer into the ghost frame; the
//    communication event then gates the compute stream. On one GPU the unpack
//    reads the neighbour's send buffer directly (the transfer is the copy
//    itself); across GPUs it would read a received copy.
//  * Each tile's sweep is the plain sweep kernel applied to a view of its
//    buffer: the view spans the owned block plus the ghost rows/columns on the
//    sides that have a neighbour, so the view's interior is exactly the
//    owned points that are interior points of the whole grid. Results are
//    bit-identical to the single-grid method.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"

namespace sten {

void launch_sweep_f64_internal(const double* in, double* out, int H, int W, int64_t ld, double c, hipStream_t s);

namespace {

struct alignas(16) Strip {
    const double* src;
    double* dst;
    int64_t src_stride;
    int64_t dst_stride;
    int32_t n, pad;
};

// Copy strips: strip s = blockIdx.y; elements by threads of blockIdx.x.
__global__ void strip_copy_kernel(const Strip* __restrict__ strips, int nstrips) {
    const int s = blockIdx.y;
    if (s >= nstrips) return;
    const Strip st = strips[s];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < st.n; k += gridDim.x * blockDim.x)
        st.dst[(int64_t)k * st.dst_stride] = st.src[(int64_t)k * st.src_stride];
}

// Global grid rows/cols [r0, r0+h) x [c0, c0+w) <-> owned block of a tile buffer.
__global__ void block_copy_kernel(const double* __restrict__ src, int64_t src_ld, double* __restrict__ d1,
                                  double* __restrict__ d2, int64_t dst_ld, int h, int w) {
    const int64_t total = (int64_t)h * w;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / w;
        const int64_t j = idx - i * w;
        const double v = src[i * src_ld + j];
        d1[i * dst_ld + j] = v;
        if (d2 != nullptr) d2[i * dst_ld + j] = v;
    }
}

struct Tile {
    int r0, c0, h, w;       // owned block in grid coordinates
    int64_t ldt;            // row stride of the tile buffers (elements, even)
    double* buf[2];         // (h + 2) x ldt each; owned (i, j) at [(i + 1) * ldt + (j + 1)]
    double* send[4];        // per edge: 0 north, 1 south, 2 west, 3 east (NULL when no neighbour)
    int nb[4];              // neighbour tile index per edge, -1 when none
};

}  // namespace
}  // namespace sten

struct sten_tiled_s {
    int64_t H = 0, W = 0;
    int pr = 0, pc = 0;
    std::vector<sten::Tile> tiles;
    sten::Strip* d_pack[2] = {nullptr, nullptr};    // per buffer
    sten::Strip* d_unpack[2] = {nullptr, nullptr};
    int n_pack = 0, n_unpack = 0, max_strip = 0;
    std::vector<sten::Strip> h_pack[2], h_unpack[2];
    int cur = 0;                 // buffer holding the current state
    int64_t local_epoch[2] = {0, 0};
    int64_t ghost_epoch[2] = {0, 0};
    int64_t n_exchanges = 0, n_skipped = 0, n_sweep_launches = 0;
    hipEvent_t ev_compute = nullptr, ev_comm = nullptr;
    bool uploaded = false;
};

namespace sten {
namespace {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte layout of the workspace: tile buffers, send buffers, then the strip tables.
struct Layout {
    std::vector<size_t> buf_off[2], send_off[4];
    size_t tables_off = 0, total = 0;
};

int split(int64_t n, int parts, int k) { return (int)((n * k) / parts); }

Layout plan_layout(int64_t H, int64_t W, int pr, int pc, std::vector<Tile>& tiles, int& nstrips) {
    Layout L;
    tiles.clear();
    size_t off = 0;
    nstrips = 0;
    for (int a = 0; a < pr; ++a) {
        for (int b = 0; b < pc; ++b) {
            Tile t{};
            t.r0 = split(H, pr, a);
            t.c0 = split(W, pc, b);
            t.h = split(H, pr, a + 1) - t.r0;
            t.w = split(W, pc, b + 1) - t.c0;
            t.ldt = (int64_t)align_up((size_t)t.w + 2, 2);
            t.nb[0] = a > 0 ? (a - 1) * pc + b : -1;
            t.nb[1] = a < pr - 1 ? (a + 1) * pc + b : -1;
            t.nb[2] = b > 0 ? a * pc + b - 1 : -1;
            t.nb[3] = b < pc - 1 ? a * pc + b + 1 : -1;
            tiles.push_back(t);
        }
    }
    for (int k = 0; k < 2; ++k) L.buf_off[k].resize(tiles.size());
    for (int e = 0; e < 4; ++e) L.send_off[e].resize(tiles.size());
    for (size_t t = 0; t < tiles.size(); ++t) {
        const Tile& T = tiles[t];
        for (int k = 0; k < 2; ++k) {
            // +2 elements of slack so the sweep view can start 16-byte aligned
            L.buf_off[k][t] = off;
            off = align_up(off + ((size_t)(T.h + 2) * T.ldt + 2) * sizeof(double), 256);
        }
        for (int e = 0; e < 4; ++e) {
            L.send_off[e][t] = off;
            if (T.nb[e] >= 0) {
                ++nstrips;
                off = align_up(off + (size_t)(e < 2 ? T.w : T.h) * sizeof(double), 256);
            }
        }
    }
    L.tables_off = off;
    off += 4 * (size_t)std::max(nstrips, 1) * sizeof(Strip);
    L.total = align_up(off, 256);
    return L;
}

// View of a tile buffer whose interior is the tile's owned grid-interior points.
struct View {
    int64_t off;  // element offset from the buffer base
    int vh, vw;   // view rows/cols
};

View tile_view(const Tile& t, int64_t H, int64_t W) {
    const int top = (t.r0 == 0) ? 1 : 0;
    const int bottom = (t.r0 + t.h == H) ? t.h : t.h + 1;
    const int left = (t.c0 == 0) ? 1 : 0;
    const int right = (t.c0 + t.w == W) ? t.w : t.w + 1;
    return View{(int64_t)top * t.ldt + left, bottom - top + 1, right - left + 1};
}

sten_status upload_tables(sten_tiled_s* p, hipStream_t s) {
    for (int k = 0; k < 2; ++k) {
        if (p->n_pack > 0) {
            hipError_t e = hipMemcpyAsync(p->d_pack[k], p->h_pack[k].data(), p->n_pack * sizeof(Strip),
                                          hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e);
            e = hipMemcpyAsync(p->d_unpack[k], p->h_unpack[k].data(), p->n_unpack * sizeof(Strip),
                               hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e);
        }
    }
    p->uploaded = true;
    return STEN_OK;
}

sten_status exchange(sten_tiled_s* p, int k, hipStream_t compute, hipStream_t comm) {
    if (p->ghost_epoch[k] == p->local_epoch[k]) {
        ++p->n_skipped;
        return STEN_OK;
    }
    if (p->n_pack > 0) {
        hipError_t e = hipEventRecord(p->ev_compute, compute);
        if (e == hipSuccess) e = hipStreamWaitEvent(comm, p->ev_compute, 0);
        if (e != hipSuccess) return hip_fail(e);
        const uint32_t gx = (uint32_t)std::min(64, std::max(1, (p->max_strip + 255) / 256));
        strip_copy_kernel<<<dim3(gx, p->n_pack), 256, 0, comm>>>(p->d_pack[k], p->n_pack);
        strip_copy_kernel<<<dim3(gx, p->n_unpack), 256, 0, comm>>>(p->d_unpack[k], p->n_unpack);
        e = hipEventRecord(p->ev_comm, comm);
        if (e == hipSuccess) e = hipStreamWaitEvent(compute, p->ev_comm, 0);
        if (e != hipSuccess) return hip_fail(e);
    }
    p->ghost_epoch[k] = p->local_epoch[k];
    ++p->n_exchanges;
    return check_launch();
}

}  // namespace
}  // namespace sten

extern "C" {

size_t sten_tiled_workspace_bytes(int64_t H, int64_t W, int32_t pr, int32_t pc) {
    if (H < 1 || W < 1 || pr < 1 || pc < 1 || pr > H || pc > W) return 0;
    std::vector<sten::Tile> tiles;
    int ns = 0;
    return sten::plan_layout(H, W, pr, pc, tiles, ns).total;
}

sten_status sten_tiled_create(int64_t H, int64_t W, int32_t pr, int32_t pc, void* dev_ws, size_t ws_bytes,
                              sten_tiled_handle* out) {
    using namespace sten;
    if (out == nullptr) return STEN_ERR_ARG;
    *out = nullptr;
    if (H < 1 || W < 1 || pr < 1 || pc < 1 || pr > H || pc > W) return STEN_ERR_ARG;
    if (H > INT32_MAX / 2 || W > INT32_MAX / 2) return STEN_ERR_ARG;
    if (dev_ws == nullptr) return STEN_ERR_PTR;
    if ((uintptr_t)dev_ws % 256 != 0) return STEN_ERR_ARG;
    auto* p = new sten_tiled_s();
    p->H = H;
    p->W = W;
    p->pr = pr;
    p->pc = pc;
    int nstrips = 0;
    Layout L = plan_layout(H, W, pr, pc, p->tiles, nstrips);
    if (ws_bytes < L.total) {
        delete p;
        return STEN_ERR_WORKSPACE;
    }
    if (!is_device_ptr(dev_ws)) {
        delete p;
        return STEN_ERR_PTR;
    }
    char* base = (char*)dev_ws;
    for (size_t t = 0; t < p->tiles.size(); ++t) {
        Tile& T = p->tiles[t];
        const View v = tile_view(T, H, W);
        for (int k = 0; k < 2; ++k) {
            // shift the buffer so that the view start lands on a 16-byte boundary
            double* b = (double*)(base + L.buf_off[k][t]);
            const int64_t mis = v.off % 2;
            T.buf[k] = b + (mis ? 1 : 0);
        }
        for (int e = 0; e < 4; ++e) T.send[e] = T.nb[e] >= 0 ? (double*)(base + L.send_off[e][t]) : nullptr;
    }
    // strip tables: pack (owned boundary -> own send buffer), unpack (neighbour's send -> own ghost)
    for (int k = 0; k < 2; ++k) {
        for (const Tile& T : p->tiles) {
            const double* own = T.buf[k] + T.ldt + 1;  // owned (0, 0)
            for (int e = 0; e < 4; ++e) {
                if (T.nb[e] < 0) continue;
                Strip s{};
                if (e == 0) s = Strip{own, T.send[e], 1, 1, T.w, 0};
                if (e == 1) s = Strip{own + (int64_t)(T.h - 1) * T.ldt, T.send[e], 1, 1, T.w, 0};
                if (e == 2) s = Strip{own, T.send[e], T.ldt, 1, T.h, 0};
                if (e == 3) s = Strip{own + (T.w - 1), T.send[e], T.ldt, 1, T.h, 0};
                p->h_pack[k].push_back(s);
                p->max_strip = std::max(p->max_strip, s.n);
            }
        }
        for (const Tile& T : p->tiles) {
            double* gb = T.buf[k];  // ghost frame: row 0, row h+1, col 0, col w+1
            for (int e = 0; e < 4; ++e) {
                if (T.nb[e] < 0) continue;
                const Tile& N = p->tiles[T.nb[e]];
                const int opp = e ^ 1;  // north <-> south, west <-> east
                Strip s{};
                if (e == 0) s = Strip{N.send[opp], gb + 1, 1, 1, T.w, 0};
                if (e == 1) s = Strip{N.send[opp], gb + (int64_t)(T.h + 1) * T.ldt + 1, 1, 1, T.w, 0};
                if (e == 2) s = Strip{N.send[opp], gb + T.ldt, 1, T.ldt, T.h, 0};
                if (e == 3) s = Strip{N.send[opp], gb + T.ldt + (T.w + 1), 1, T.ldt, T.h, 0};
                p->h_unpack[k].push_back(s);
            }
        }
    }
    p->n_pack = (int)p->h_pack[0].size();
    p->n_unpack = (int)p->h_unpack[0].size();
    Strip* tables = (Strip*)(base + L.tables_off);
    const int n = std::max(nstrips, 1);
    p->d_pack[0] = tables;
    p->d_pack[1] = tables + n;
    p->d_unpack[0] = tables + 2 * n;
    p->d_unpack[1] = tables + 3 * n;
    hipError_t e = hipEventCreateWithFlags(&p->ev_compute, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_comm, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (p->ev_compute) (void)hipEventDestroy(p->ev_compute);
        delete p;
        return hip_fail(e);
    }
    *out = p;
    return STEN_OK;
}

sten_status sten_tiled_scatter(sten_tiled_handle p, const double* u, int64_t ld, hipStream_t stream) {
    using namespace sten;
    if (p == nullptr) return STEN_ERR_ARG;
    if (ld < p->W) return STEN_ERR_ARG;
    if (u == nullptr) return STEN_ERR_PTR;
    if (!is_device_ptr(u)) return STEN_ERR_PTR;
    if (!p->uploaded) {
        sten_status st = upload_tables(p, stream);
        if (st != STEN_OK) return st;
    }
    for (const Tile& T : p->tiles) {
        const int64_t total = (int64_t)T.h * T.w;
        const uint32_t blocks = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
        block_copy_kernel<<<blocks, 256, 0, stream>>>(u + (int64_t)T.r0 * ld + T.c0, ld, T.buf[0] + T.ldt + 1,
                                                      T.buf[1] + T.ldt + 1, T.ldt, T.h, T.w);
    }
    p->cur = 0;
    ++p->local_epoch[0];
    ++p->local_epoch[1];
    return check_launch();
}

sten_status sten_tiled_gather(sten_tiled_handle p, double* u, int64_t ld, hipStream_t stream) {
    using namespace sten;
    if (p == nullptr) return STEN_ERR_ARG;
    if (ld < p->W) return STEN_ERR_ARG;
    if (u == nullptr) return STEN_ERR_PTR;
    if (!is_device_ptr(u)) return STEN_ERR_PTR;
    for (const Tile& T : p->tiles) {
        const int64_t total = (int64_t)T.h * T.w;
        const uint32_t blocks = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
        block_copy_kernel<<<blocks, 256, 0, stream>>>(T.buf[p->cur] + T.ldt + 1, T.ldt,
                                                      u + (int64_t)T.r0 * ld + T.c0, nullptr, ld, T.h, T.w);
    }
    return check_launch();
}

sten_status sten_tiled_exchange(sten_tiled_handle p, hipStream_t compute, hipStream_t comm) {
    if (p == nullptr) return STEN_ERR_ARG;
    if (!p->uploaded) {
        sten_status st = sten::upload_tables(p, compute);
        if (st != STEN_OK) return st;
    }
    return sten::exchange(p, p->cur, compute, comm);
}

sten_status sten_tiled_run(sten_tiled_handle p, int32_t T, double c, hipStream_t compute, hipStream_t comm) {
    using namespace sten;
    if (p == nullptr || T < 0) return STEN_ERR_ARG;
    if (!p->uploaded) {
        sten_status st = upload_tables(p, compute);
        if (st != STEN_OK) return st;
    }
    for (int32_t k = 0; k < T; ++k) {
        const int src = p->cur, dst = 1 - p->cur;
        sten_status st = exchange(p, src, compute, comm);
        if (st != STEN_OK) return st;
        for (const Tile& t : p->tiles) {
            const View v = tile_view(t, p->H, p->W);
            if (v.vh < 3 || v.vw < 3) continue;
            launch_sweep_f64_internal(t.buf[src] + v.off, t.buf[dst] + v.off, v.vh, v.vw, t.ldt, c, compute);
            ++p->n_sweep_launches;
        }
        ++p->local_epoch[dst];
        p->cur = dst;
    }
    return check_launch();
}

sten_status sten_tiled_stats(sten_tiled_handle p, int64_t* stats, int32_t n) {
    if (p == nullptr || stats == nullptr || n < 5) return STEN_ERR_ARG;
    stats[0] = (int64_t)p->tiles.size();
    stats[1] = p->n_exchanges;
    stats[2] = p->n_skipped;
    stats[3] = p->n_sweep_launches;
    stats[4] = p->n_pack;
    return STEN_OK;
}

sten_status sten_tiled_destroy(sten_tiled_handle p) {
    if (p == nullptr) return STEN_OK;
    if (p->ev_compute) (void)hipEventDestroy(p->ev_compute);
    if (p->ev_comm) (void)hipEventDestroy(p->ev_comm);
    delete p;
    return STEN_OK;
}

}  // extern "C"
