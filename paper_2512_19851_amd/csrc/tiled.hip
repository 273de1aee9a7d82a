// Tiled execution of the FP64 method on one GPU: the paper's chare layout and
// DAG-node execution (Section III-C, data layout and DAG execution), with all
// tiles on one device.
//
//  * The H x W grid is split into pr x pc tiles ("chares"). Each tile holds
//    its owned block plus a ghost frame of depth g on every side, in two
//    buffers (the ping-pong pair). g = 1 is the ghost depth of the five-point
//    stencil; a deeper frame lets a tile run up to g sweeps between exchanges.
//  * Before a sweep reads an array, its ghosts are refreshed if the array's
//    local generation epoch differs from its ghost epoch: on the
//    communication stream, after waiting for the compute event, the exchange
//    kernels run, and the communication event then gates the compute stream
//    (no events when the two streams are the same).
//  * Exchange modes. Packed (the paper's scheme): a pack kernel copies each
//    tile's boundary blocks into one send buffer per neighbour and an unpack
//    kernel copies each neighbour's send buffer into the ghost frame; on one
//    GPU the unpack reads the neighbour's send buffer directly (the transfer
//    is the copy itself), across GPUs it would read a received copy. Direct:
//    one kernel copies each neighbour's boundary block straight into the ghost
//    frame, as a peer store into the neighbour's memory would.
//  * g sweeps depend on the diagonal neighbours too (the cone of g sweeps of a
//    five-point stencil is a diamond of radius g), so for g > 1 the exchange
//    also carries the g x g corner blocks between diagonal neighbours. For
//    g = 1 the corners are never read.
//  * Each tile sweeps a view of its buffer: the owned block plus the whole
//    ghost frame on the sides that have a neighbour. On a side without one the
//    view ends at the owned boundary row or column, which is the grid's fixed
//    ring. A sweep of the view leaves the view's own ring unchanged, so after
//    s <= g sweeps a point at distance d from a ghost side is exact when
//    d >= s: every owned point is. Results are bit-identical to the
//    single-grid method. Chunks of one sweep use one launch of the one-sweep
//    kernel over all tile views, chunks of s > 1 sweeps one launch of the
//    streaming blocked kernel over all tile views.
//  * Direct mode at depth 1 does the exchange inside the sweep: the sweep also
//    stores each tile's first and last interior rows and columns into its
//    neighbours' ghost cells of the buffer it writes (except in a run's last
//    sweep), so one launch per sweep remains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"

namespace sten {

void launch_sweep_f64_internal(const double* in, double* out, int H, int W, int64_t ld, double c, hipStream_t s);

constexpr int kMaxGhost = 12;
// Most tiles per tiling: the plan keeps host tables per tile and per message,
// so an unbounded count would let a caller's sizes exhaust host memory.
constexpr int64_t kMaxTiles = (int64_t)1 << 16;

namespace {

// A rows x cols rectangle copy between two row-major regions.
struct alignas(16) Strip {
    const double* src;
    double* dst;
    int64_t src_ld;
    int64_t dst_ld;
    int32_t rows, cols;
};

// Copy strips: strip s = blockIdx.y; its elements by the threads of blockIdx.x.
__global__ void strip_copy_kernel(const Strip* __restrict__ strips, int nstrips) {
    const int s = blockIdx.y;
    if (s >= nstrips) return;
    const Strip st = strips[s];
    const int64_t total = (int64_t)st.rows * st.cols;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = k / st.cols;
        const int64_t j = k - i * st.cols;
        st.dst[i * st.dst_ld + j] = st.src[i * st.src_ld + j];
    }
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

// Neighbour directions: 0 north, 1 south, 2 west, 3 east, 4 north-west,
// 5 north-east, 6 south-west, 7 south-east (north = lower row index).
constexpr int kDirs = 8;
constexpr int kDirRow[kDirs] = {-1, 1, 0, 0, -1, -1, 1, 1};
constexpr int kDirCol[kDirs] = {0, 0, -1, 1, -1, 1, -1, 1};
constexpr int kOpposite[kDirs] = {1, 0, 3, 2, 7, 6, 5, 4};

struct Tile {
    int r0, c0, h, w;       // owned block in grid coordinates
    int64_t ldt;            // row stride of the tile buffers (elements, even)
    double* buf[2];         // (h + 2g) x ldt each; owned (i, j) at [(i + g) * ldt + (j + g)]
    double* send[kDirs];    // packed mode: send buffer per neighbour (NULL when none)
    int nb[kDirs];          // neighbour tile index per direction, -1 when none
};

}  // namespace
}  // namespace sten

struct sten_tiled_s {
    int64_t H = 0, W = 0;
    int pr = 0, pc = 0, g = 1;
    int mode = 0;  // 0: packed (pack + unpack through send buffers), 1: direct
    std::vector<sten::Tile> tiles;
    // per buffer k: the copy tables of one exchange (packed: pack then unpack; direct: copy)
    std::vector<sten::Strip> h_pack[2], h_unpack[2];
    sten::Strip* d_pack[2] = {nullptr, nullptr};
    sten::Strip* d_unpack[2] = {nullptr, nullptr};
    int n_strips = 0;                 // messages per exchange
    int64_t max_strip = 0;            // largest message (elements; g x a tile side can pass 2^31)
    int cur = 0;                      // buffer holding the current state
    int64_t local_epoch[2] = {0, 0};
    int64_t ghost_epoch[2] = {0, 0};
    int64_t n_exchanges = 0, n_skipped = 0, n_sweep_launches = 0;
    hipEvent_t ev_compute = nullptr, ev_comm = nullptr;
    bool uploaded = false;
};

namespace sten {
namespace {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int split(int64_t n, int parts, int k) { return (int)((n * k) / parts); }

// A region of the workspace (bytes from its base).
struct Region {
    size_t off, bytes;
};

// Byte layout of the workspace: tile buffers, send buffers, then the strip tables.
struct Layout {
    std::vector<size_t> buf_off[2], send_off;  // send_off[tile * 8 + direction]
    std::vector<Region> regions;  // every buffer, for the bounds check
    size_t buf_bytes_total = 0;
    size_t tables_off = 0, table_slots = 0, total = 0;
};

// Tiles of the H x W grid, or an empty vector if the tiling is invalid for ghost depth g:
// a tile must be at least g deep across every edge it shares with a neighbour.
std::vector<Tile> make_tiles(int64_t H, int64_t W, int pr, int pc, int g) {
    std::vector<Tile> tiles;
    if (H < 1 || W < 1 || pr < 1 || pc < 1 || pr > H || pc > W || g < 1 || g > kMaxGhost) return tiles;
    if ((int64_t)pr * pc > kMaxTiles) return tiles;
    if (H > INT32_MAX / 2 || W > INT32_MAX / 2) return tiles;
    for (int a = 0; a < pr; ++a) {
        for (int b = 0; b < pc; ++b) {
            Tile t{};
            t.r0 = split(H, pr, a);
            t.c0 = split(W, pc, b);
            t.h = split(H, pr, a + 1) - t.r0;
            t.w = split(W, pc, b + 1) - t.c0;
            if ((pr > 1 && t.h < g) || (pc > 1 && t.w < g)) return {};
            t.ldt = (int64_t)align_up((size_t)t.w + 2 * g, 2);
            for (int d = 0; d < kDirs; ++d) {
                const int na = a + kDirRow[d], nbc = b + kDirCol[d];
                const bool corner = kDirRow[d] != 0 && kDirCol[d] != 0;
                // corner blocks are read only by chunks of more than one sweep
                const bool used = !corner || g > 1;
                t.nb[d] = (used && na >= 0 && na < pr && nbc >= 0 && nbc < pc) ? na * pc + nbc : -1;
            }
            tiles.push_back(t);
        }
    }
    return tiles;
}

// A rectangle of a tile buffer (buffer rows/cols).
struct Rect {
    int row, col, rows, cols;
};

// The g-deep block of tile t's owned points next to its side or corner d.
Rect owned_block(const Tile& t, int d, int g) {
    Rect r{};
    r.row = kDirRow[d] < 0 ? g : (kDirRow[d] > 0 ? t.h : g);
    r.rows = kDirRow[d] == 0 ? t.h : g;
    r.col = kDirCol[d] < 0 ? g : (kDirCol[d] > 0 ? t.w : g);
    r.cols = kDirCol[d] == 0 ? t.w : g;
    return r;
}

// The part of tile t's ghost frame on its side or corner d.
Rect ghost_block(const Tile& t, int d, int g) {
    Rect r{};
    r.row = kDirRow[d] < 0 ? 0 : (kDirRow[d] > 0 ? g + t.h : g);
    r.rows = kDirRow[d] == 0 ? t.h : g;
    r.col = kDirCol[d] < 0 ? 0 : (kDirCol[d] > 0 ? g + t.w : g);
    r.cols = kDirCol[d] == 0 ? t.w : g;
    return r;
}

Layout plan_layout(const std::vector<Tile>& tiles, int g, int mode) {
    Layout L;
    size_t off = 0;
    int nstrips = 0;
    for (int k = 0; k < 2; ++k) L.buf_off[k].resize(tiles.size());
    L.send_off.assign(tiles.size() * kDirs, 0);
    for (size_t t = 0; t < tiles.size(); ++t) {
        const Tile& T = tiles[t];
        for (int k = 0; k < 2; ++k) {
            // +2 elements of slack so the sweep view can start 16-byte aligned
            const size_t bytes = ((size_t)(T.h + 2 * g) * T.ldt + 2) * sizeof(double);
            L.buf_off[k][t] = off;
            L.regions.push_back(Region{off, bytes});
            off = align_up(off + bytes, 256);
        }
        for (int d = 0; d < kDirs; ++d) {
            if (T.nb[d] < 0) continue;
            ++nstrips;
            if (mode != 0) continue;
            const Rect r = owned_block(T, d, g);
            const size_t bytes = (size_t)r.rows * r.cols * sizeof(double);
            L.send_off[t * kDirs + d] = off;
            L.regions.push_back(Region{off, bytes});
            off = align_up(off + bytes, 256);
        }
    }
    L.tables_off = off;
    // 2 buffers x 2 tables, each sized for every message of an exchange
    L.table_slots = (size_t)std::max(nstrips, 1);
    off += 4 * L.table_slots * sizeof(Strip);
    L.total = align_up(off, 256);
    return L;
}

// View of a tile buffer: the owned block plus the ghost frame on the sides that have a neighbour.
struct View {
    int64_t off;  // element offset from the buffer base
    int vh, vw;   // view rows/cols
};

View tile_view(const Tile& t, int g) {
    const int top = t.nb[0] >= 0 ? 0 : g;
    const int bottom = t.nb[1] >= 0 ? t.h + 2 * g : t.h + g;
    const int left = t.nb[2] >= 0 ? 0 : g;
    const int right = t.nb[3] >= 0 ? t.w + 2 * g : t.w + g;
    return View{(int64_t)top * t.ldt + left, bottom - top, right - left};
}

double* at(const Tile& t, int k, const Rect& r) { return t.buf[k] + (int64_t)r.row * t.ldt + r.col; }

// Fill tile pointers and copy tables for a workspace at `base` (pointers are only computed here).
void build_plan(sten_tiled_s* p, const Layout& L, char* base) {
    const int g = p->g;
    for (size_t t = 0; t < p->tiles.size(); ++t) {
        Tile& T = p->tiles[t];
        const View v = tile_view(T, g);
        for (int k = 0; k < 2; ++k) {
            // shift the buffer so that the view start lands on a 16-byte boundary
            double* b = (double*)(base + L.buf_off[k][t]);
            T.buf[k] = b + (v.off % 2 ? 1 : 0);
        }
        for (int d = 0; d < kDirs; ++d)
            T.send[d] = (p->mode == 0 && T.nb[d] >= 0) ? (double*)(base + L.send_off[t * kDirs + d]) : nullptr;
    }
    p->max_strip = 0;
    for (int k = 0; k < 2; ++k) {
        p->h_pack[k].clear();
        p->h_unpack[k].clear();
        for (const Tile& T : p->tiles) {
            for (int d = 0; d < kDirs; ++d) {
                if (T.nb[d] < 0) continue;
                const Tile& N = p->tiles[T.nb[d]];
                const Rect src = owned_block(N, kOpposite[d], g);  // what the neighbour sends toward T
                const Rect dst = ghost_block(T, d, g);
                if (p->mode == 0) {
                    // the neighbour packs its block into its send buffer toward T; T unpacks it
                    double* sb = N.send[kOpposite[d]];
                    p->h_pack[k].push_back(Strip{at(N, k, src), sb, N.ldt, src.cols, src.rows, src.cols});
                    p->h_unpack[k].push_back(Strip{sb, at(T, k, dst), src.cols, T.ldt, dst.rows, dst.cols});
                } else {
                    p->h_pack[k].push_back(Strip{at(N, k, src), at(T, k, dst), N.ldt, T.ldt, dst.rows, dst.cols});
                }
                p->max_strip = std::max(p->max_strip, (int64_t)dst.rows * dst.cols);
            }
        }
    }
    p->n_strips = (int)p->h_pack[0].size();
    Strip* tables = (Strip*)(base + L.tables_off);
    for (int k = 0; k < 2; ++k) {
        p->d_pack[k] = tables + (size_t)(2 * k) * L.table_slots;
        p->d_unpack[k] = tables + (size_t)(2 * k + 1) * L.table_slots;
    }
}

// True if [ptr, ptr + bytes) lies inside one region of the workspace at `base`.
bool inside(const Layout& L, const char* base, const void* ptr, size_t bytes) {
    const char* q = (const char*)ptr;
    if (q < base) return false;
    const size_t off = (size_t)(q - base);
    for (const Region& r : L.regions)
        if (off >= r.off && off + bytes <= r.off + r.bytes) return true;
    return false;
}

size_t rect_bytes(int64_t rows, int64_t cols, int64_t ld) {
    return rows <= 0 || cols <= 0 ? 0 : (size_t)((rows - 1) * ld + cols) * sizeof(double);
}

// Host check that every copy and every sweep view stays inside its buffer, that a
// message and its ghost block agree in shape, and that views are 16-byte aligned.
bool plan_in_bounds(const sten_tiled_s* p, const Layout& L, const char* base) {
    for (int k = 0; k < 2; ++k) {
        if (p->h_pack[k].size() > L.table_slots) return false;
        if (p->mode == 0 && p->h_unpack[k].size() != p->h_pack[k].size()) return false;
        if (p->mode != 0 && !p->h_unpack[k].empty()) return false;
        for (const auto* tab : {&p->h_pack[k], &p->h_unpack[k]}) {
            for (const Strip& s : *tab) {
                if (s.rows < 1 || s.cols < 1 || s.cols > s.src_ld || s.cols > s.dst_ld) return false;
                if (!inside(L, base, s.src, rect_bytes(s.rows, s.cols, s.src_ld))) return false;
                if (!inside(L, base, s.dst, rect_bytes(s.rows, s.cols, s.dst_ld))) return false;
            }
        }
        for (size_t i = 0; i < p->h_unpack[k].size(); ++i) {
            const Strip& a = p->h_pack[k][i];
            const Strip& b = p->h_unpack[k][i];
            if (a.dst != b.src || a.rows != b.rows || a.cols != b.cols) return false;
        }
    }
    for (const Tile& T : p->tiles) {
        const View v = tile_view(T, p->g);
        if (v.vw > T.ldt) return false;
        for (int k = 0; k < 2; ++k) {
            const double* a = T.buf[k] + v.off;
            if (!inside(L, base, a, rect_bytes(v.vh, v.vw, T.ldt))) return false;
            if ((size_t)((const char*)a - base) % 16 != 0) return false;
            // the owned block (scatter and gather)
            if (!inside(L, base, T.buf[k] + (int64_t)p->g * T.ldt + p->g, rect_bytes(T.h, T.w, T.ldt)))
                return false;
        }
    }
    return true;
}

sten_status upload_tables(sten_tiled_s* p, hipStream_t s) {
    for (int k = 0; k < 2; ++k) {
        for (int u = 0; u < 2; ++u) {
            const std::vector<Strip>& h = u ? p->h_unpack[k] : p->h_pack[k];
            if (h.empty()) continue;
            hipError_t e = hipMemcpyAsync(u ? p->d_unpack[k] : p->d_pack[k], h.data(), h.size() * sizeof(Strip),
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
    if (p->n_strips > 0) {
        const bool two = comm != compute;
        hipError_t e = hipSuccess;
        if (two) {
            e = hipEventRecord(p->ev_compute, compute);
            if (e == hipSuccess) e = hipStreamWaitEvent(comm, p->ev_compute, 0);
            if (e != hipSuccess) return hip_fail(e);
        }
        const uint32_t gx = (uint32_t)std::min<int64_t>(64, std::max<int64_t>(1, (p->max_strip + 255) / 256));
        const int n = p->n_strips;
        strip_copy_kernel<<<dim3(gx, n), 256, 0, comm>>>(p->d_pack[k], n);
        if (p->mode == 0) strip_copy_kernel<<<dim3(gx, n), 256, 0, comm>>>(p->d_unpack[k], n);
        if (two) {
            e = hipEventRecord(p->ev_comm, comm);
            if (e == hipSuccess) e = hipStreamWaitEvent(compute, p->ev_comm, 0);
            if (e != hipSuccess) return hip_fail(e);
        }
    }
    p->ghost_epoch[k] = p->local_epoch[k];
    ++p->n_exchanges;
    return check_launch();
}

// The ghost cells of neighbour nb's view in buffer k at its view row `row` (north/south) or column
// `col` (west/east), -1 selecting the last one.
double* ghost_line(const sten_tiled_s* p, int nb, int k, int row, int col) {
    const Tile& u = p->tiles[nb];
    const View nv = tile_view(u, p->g);
    const int r = row < 0 ? nv.vh - 1 : row, cc = col < 0 ? nv.vw - 1 : col;
    return u.buf[k] + nv.off + (int64_t)r * u.ldt + cc;
}

// s sweeps of every tile from buffer src to buffer 1 - src: one sweep as one
// launch of the single-sweep kernel over all tiles (per 32 tiles), several as
// one launch of the streaming blocked kernel over all tiles (per 32 tiles).
// fuse (depth 1, one sweep): the sweep also stores every tile's edge rows and
// columns into its neighbours' ghost cells in buffer 1 - src, which is then a
// complete exchange. Returns whether it did.
bool sweep_tiles(sten_tiled_s* p, int src, int s, double c, hipStream_t compute, bool fuse) {
    const int dst = 1 - src;
    std::vector<GridView<double>> views;
    std::vector<GridMirror> mirrors;
    // a tile whose view is under 3 x 3 has no interior point and is not swept, so it would not
    // refresh its neighbours' ghost copies of its values in buffer dst: no fused exchange then
    for (const Tile& t : p->tiles) {
        const View v = tile_view(t, p->g);
        if (v.vh < 3 || v.vw < 3) fuse = false;
    }
    for (const Tile& t : p->tiles) {
        const View v = tile_view(t, p->g);
        if (v.vh < 3 || v.vw < 3) continue;
        views.push_back(GridView<double>{t.buf[src] + v.off, t.buf[dst] + v.off, v.vh, v.vw, t.ldt});
        if (fuse) {
            GridMirror m;
            if (t.nb[0] >= 0) m.north = ghost_line(p, t.nb[0], dst, -1, 0);
            if (t.nb[1] >= 0) m.south = ghost_line(p, t.nb[1], dst, 0, 0);
            if (t.nb[2] >= 0) {
                m.west = ghost_line(p, t.nb[2], dst, 0, -1);
                m.ld_west = p->tiles[t.nb[2]].ldt;
            }
            if (t.nb[3] >= 0) {
                m.east = ghost_line(p, t.nb[3], dst, 0, 0);
                m.ld_east = p->tiles[t.nb[3]].ldt;
            }
            mirrors.push_back(m);
        }
    }
    if (views.empty()) return false;
    const int64_t launches = ((int64_t)views.size() + kMaxStreamGridsPerLaunch - 1) / kMaxStreamGridsPerLaunch;
    if (s == 1) {
        if (launch_sweep_grids_f64(views.data(), (int)views.size(), c, compute, fuse ? mirrors.data() : nullptr)) {
            p->n_sweep_launches += launches;
            return fuse;
        }
        // a view off the 16-byte alignment the plan lays out: one launch per tile, no fused exchange
        for (const GridView<double>& v : views) {
            launch_sweep_f64_internal(v.in, v.out, v.H, v.W, v.ld, c, compute);
            ++p->n_sweep_launches;
        }
        return false;
    }
    launch_stream_grids_f64(views.data(), (int)views.size(), c, s, compute);
    p->n_sweep_launches += launches;
    return false;
}

sten_status make_plan(int64_t H, int64_t W, int pr, int pc, int g, int mode, sten_tiled_s* p, Layout& L) {
    if (mode != 0 && mode != 1) return STEN_ERR_ARG;
    p->tiles = make_tiles(H, W, pr, pc, g);
    if (p->tiles.empty()) return STEN_ERR_ARG;
    // the streaming kernel addresses a row with 32-bit byte offsets
    if (g > 1 && (W + 2 * g) * (int64_t)sizeof(double) >= ((int64_t)1 << 30)) return STEN_ERR_UNSUPPORTED;
    p->H = H;
    p->W = W;
    p->pr = pr;
    p->pc = pc;
    p->g = g;
    p->mode = mode;
    L = plan_layout(p->tiles, g, mode);
    return STEN_OK;
}

}  // namespace
}  // namespace sten

extern "C" {

size_t sten_tiled_workspace_bytes_ex(int64_t H, int64_t W, int32_t pr, int32_t pc, int32_t ghost, int32_t mode) {
    sten_tiled_s plan;
    sten::Layout L;
    if (sten::make_plan(H, W, pr, pc, ghost, mode, &plan, L) != STEN_OK) return 0;
    return L.total;
}

size_t sten_tiled_workspace_bytes(int64_t H, int64_t W, int32_t pr, int32_t pc) {
    return sten_tiled_workspace_bytes_ex(H, W, pr, pc, 1, STEN_TILED_PACKED);
}

sten_status sten_tiled_plan_check(int64_t H, int64_t W, int32_t pr, int32_t pc, int32_t ghost, int32_t mode,
                                  int64_t* info, int32_t n) {
    using namespace sten;
    if (info == nullptr || n < 4) return STEN_ERR_ARG;
    sten_tiled_s plan;
    Layout L;
    const sten_status st = make_plan(H, W, pr, pc, ghost, mode, &plan, L);
    if (st != STEN_OK) return st;
    // a stand-in base address: pointers are computed, never dereferenced
    char* base = (char*)(uintptr_t)((uint64_t)1 << 40);
    build_plan(&plan, L, base);
    info[0] = (int64_t)plan.tiles.size();
    info[1] = plan.n_strips;
    info[2] = plan.n_strips > 0 ? (mode == STEN_TILED_PACKED ? 2 : 1) : 0;
    info[3] = (int64_t)L.total;
    return plan_in_bounds(&plan, L, base) ? STEN_OK : STEN_ERR_UNSUPPORTED;
}

sten_status sten_tiled_create_ex(int64_t H, int64_t W, int32_t pr, int32_t pc, int32_t ghost, int32_t mode,
                                 void* dev_ws, size_t ws_bytes, sten_tiled_handle* out) {
    using namespace sten;
    if (out == nullptr) return STEN_ERR_ARG;
    *out = nullptr;
    auto* p = new sten_tiled_s();
    Layout L;
    sten_status st = make_plan(H, W, pr, pc, ghost, mode, p, L);
    if (st == STEN_OK && dev_ws == nullptr) st = STEN_ERR_PTR;
    if (st == STEN_OK && (uintptr_t)dev_ws % 256 != 0) st = STEN_ERR_ARG;
    if (st == STEN_OK && ws_bytes < L.total) st = STEN_ERR_WORKSPACE;
    if (st == STEN_OK && !is_device_ptr(dev_ws)) st = STEN_ERR_PTR;
    if (st == STEN_OK) {
        build_plan(p, L, (char*)dev_ws);
        if (!plan_in_bounds(p, L, (const char*)dev_ws)) st = STEN_ERR_UNSUPPORTED;
    }
    if (st == STEN_OK) {
        hipError_t e = hipEventCreateWithFlags(&p->ev_compute, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_comm, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (p->ev_compute) (void)hipEventDestroy(p->ev_compute);
            st = hip_fail(e);
        }
    }
    if (st != STEN_OK) {
        delete p;
        return st;
    }
    *out = p;
    return STEN_OK;
}

sten_status sten_tiled_create(int64_t H, int64_t W, int32_t pr, int32_t pc, void* dev_ws, size_t ws_bytes,
                              sten_tiled_handle* out) {
    return sten_tiled_create_ex(H, W, pr, pc, 1, STEN_TILED_PACKED, dev_ws, ws_bytes, out);
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
    const int g = p->g;
    for (const Tile& T : p->tiles) {
        const int64_t total = (int64_t)T.h * T.w;
        const uint32_t blocks = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
        block_copy_kernel<<<blocks, 256, 0, stream>>>(u + (int64_t)T.r0 * ld + T.c0, ld,
                                                      T.buf[0] + (int64_t)g * T.ldt + g,
                                                      T.buf[1] + (int64_t)g * T.ldt + g, T.ldt, T.h, T.w);
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
    const int g = p->g;
    for (const Tile& T : p->tiles) {
        const int64_t total = (int64_t)T.h * T.w;
        const uint32_t blocks = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
        block_copy_kernel<<<blocks, 256, 0, stream>>>(T.buf[p->cur] + (int64_t)g * T.ldt + g, T.ldt,
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
    if (T == 0) return STEN_OK;
    // chunks of at most g sweeps between exchanges, split as evenly as the chunk count allows
    const int chunks = (T + p->g - 1) / p->g;
    const int base = T / chunks, extra = T % chunks;
    bool fresh = false;  // the previous sweep did the exchange of the buffer it wrote
    for (int k = 0; k < chunks; ++k) {
        const int src = p->cur, dst = 1 - p->cur;
        if (!fresh) {
            sten_status st = exchange(p, src, compute, comm);
            if (st != STEN_OK) return st;
        }
        // direct mode at depth 1 stores the edge values into the neighbours' ghosts within the sweep
        // (as a peer store across GPUs would), except in the run's last sweep, whose ghosts the next
        // exchange refreshes when they are read
        const bool fuse = p->mode == 1 && p->g == 1 && k + 1 < chunks;
        fresh = sweep_tiles(p, src, base + (k < extra ? 1 : 0), c, compute, fuse);
        ++p->local_epoch[dst];
        if (fresh) {
            p->ghost_epoch[dst] = p->local_epoch[dst];
            ++p->n_exchanges;
        }
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
    stats[4] = p->n_strips;
    if (n >= 6) stats[5] = p->g;
    if (n >= 7) stats[6] = p->mode;
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
