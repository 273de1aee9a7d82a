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
#include <atomic>

#include "common.hpp"
#include "stream_common.hpp"

namespace sten {
namespace {

using namespace stream;

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

// Streaming form of the same blocking. One wave owns a strip of 64*V - 2*HALO
// output columns and a band of output rows [rb, re), and walks along the band
// once: it loads one row per step (level 0) and, for s = 1..TL, computes level
// s of the row s behind the loaded one from the last two level-(s-1) rows it
// keeps and the level-(s-1) row just produced. Level TL of the row TL behind
// is stored. Unlike the register tile above, no row is computed twice except
// the TL*(TL-1) rows a band start needs; horizontal neighbours come from DPP
// lane shifts (no LDS); interior strips skip every column test, and row tests
// run only where a level's row can leave the interior.
//
// Even bands walk down, odd bands walk up, so the 2*TL rows two neighbouring
// bands both load are loaded by both near the end (or both near the start) of
// their walks, and the second load finds many of them still in L2 (measured:
// the fetch excess falls by about half). Direction does not change a bit: the
// sum starts with N + S, and IEEE addition is commutative.
//
// Rows that a level computes before its inputs are complete (the first 2s
// steps of level s) are never read by a stored value: level s+1 first reads
// level s at step 2s+2, by which time the two rows it keeps were produced at
// steps 2s and 2s+1, the first steps where level s is complete. The prologue
// skips those levels outright. Rows outside the grid are loaded clamped to the
// grid: their values never reach an interior point (an interior row r reads
// rows r-1 and r+1 only, both inside the grid), so no branch is needed.

// Strip kinds: EDGE 0, a strip whose loaded columns are all interior (no
// column test at all); EDGE 1, a strip that touches the grid's first or last
// column but loads only columns inside the grid (the two boundary columns keep
// their value by a select, and stores are whole vectors: a boundary column is
// stored with its unchanged input value, which the output already holds);
// EDGE 2, a strip whose loads may leave the grid (columns clamped, stored
// column by column).

// One level of one row: res = c * (((N + S) + W) + E) where the row is
// interior, else the centre value (boundary ring and outside points keep it).
// `a` and `b` are the two vertical neighbours (N and S in either order).
template <typename T, int V, int EDGE>
__device__ __forceinline__ void stream_level(const T (&a)[V], const T (&m)[V], const T (&b)[V], T (&res)[V], T c,
                                             bool row_in, const bool (&col_in)[V]) {
    if (!row_in) {
#pragma unroll
        for (int e = 0; e < V; ++e) res[e] = m[e];
        return;
    }
    const T lft = lane_from_lower(m[V - 1]);  // column j0 - 1
    const T rgt = lane_from_upper(m[0]);      // column j0 + V
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const T west = (e == 0) ? lft : m[e > 0 ? e - 1 : 0];
        const T east = (e == V - 1) ? rgt : m[e < V - 1 ? e + 1 : 0];
        T sum = a[e] + b[e];
        sum = sum + west;
        sum = sum + east;
        const T v = c * sum;
        res[e] = (EDGE == 0 || col_in[e]) ? v : m[e];
    }
}

// One step: the level-0 row L (x) enters; levels 1..NACT advance by one row
// each (level s produces row L - dir*s). Level 1 reads the input rows of the
// last three steps (a0, b0, x: oldest first) straight from the load ring;
// w0[k], w1[k] hold the two latest rows of level k >= 1, older first. With
// NACT == TL the level-TL row goes to `top`.
template <typename T, int V, int TL, int NACT, int EDGE, bool ROWCHK>
__device__ __forceinline__ void stream_step(T (&w0)[TL][V], T (&w1)[TL][V], const T (&a0)[V], const T (&b0)[V],
                                            const T (&x)[V], T (&top)[V], int L, int dir, int H, T c,
                                            const bool (&col_in)[V]) {
    if constexpr (NACT >= 1) {
        T cur[V];
        stream_level<T, V, EDGE>(a0, b0, x, cur, c, !ROWCHK || (L - dir >= 1 && L - dir <= H - 2), col_in);
#pragma unroll
        for (int s = 2; s <= NACT; ++s) {
            const int r = L - dir * s;
            const bool row_in = !ROWCHK || (r >= 1 && r <= H - 2);
            T nv[V];
            stream_level<T, V, EDGE>(w0[s - 1], w1[s - 1], cur, nv, c, row_in, col_in);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                w0[s - 1][e] = w1[s - 1][e];
                w1[s - 1][e] = cur[e];
                cur[e] = nv[e];
            }
        }
        if constexpr (NACT < TL) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                w0[NACT][e] = w1[NACT][e];
                w1[NACT][e] = cur[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) top[e] = cur[e];
        }
    }
}

// Load ring: P = A + 2 slots; step t reads its row from slot t % P and, once
// done, loads the row of step t + A into slot (t + A) % P, which held the row
// of step t - 2, last read by this very step. A loaded row is therefore waited
// for A steps after its load was issued.
template <int A>
struct Ring {
    static constexpr int P = A + 2;
    static constexpr int U = (P % 3 == 0) ? P : 3 * P;  // steps per group: whole periods of every rotation
};

// Steps 0 .. 2*TL-1: level s is complete from step 2s on.
template <typename T, int V, int TL, int A, int K, int EDGE>
__device__ __forceinline__ void stream_prologue(T (&w0)[TL][V], T (&w1)[TL][V], T (&ring)[Ring<A>::P][V],
                                                const T* __restrict__ in, int L0, int dir, int H, int W, int64_t ld,
                                                int j0, T c, const bool (&col_in)[V]) {
    constexpr int P = Ring<A>::P;
    if constexpr (K < 2 * TL) {
        T unused[V];
        stream_step<T, V, TL, K / 2, EDGE, true>(w0, w1, ring[(K + P - 2) % P], ring[(K + P - 1) % P], ring[K % P],
                                                   unused, L0 + dir * K, dir, H, c, col_in);
        stream_load<T, V, EDGE>(in, L0 + dir * (K + A), H, W, ld, j0, ring[(K + A) % P]);
        __builtin_amdgcn_sched_barrier(0);
        stream_prologue<T, V, TL, A, K + 1, EDGE>(w0, w1, ring, in, L0, dir, H, W, ld, j0, c, col_in);
    }
}

// Every register rotation has a period dividing U: the ring (P) and each
// level's two kept rows plus its new row (3). An unrolled group of U steps
// therefore ends with every row back in the register it started in: no
// copies, and no wait on a load other than the one a step reads.
//
// Wave priority follows progress: a wave starts at priority 3 and drops one
// level after each quarter of its band. The hardware issues the oldest wave of
// the highest priority first, so without this the oldest wave on a SIMD ran
// ahead and the youngest finished its band alone, latency-bound; with it the
// waves sharing a SIMD advance together and finish together.
template <typename T, int V, int TL, int A, int EDGE>
__device__ __forceinline__ void stream_band(const T* __restrict__ in, T* __restrict__ out, int H, int W, int64_t ld,
                                            T c, int cs, int olo, int ohi, int rb, int re, int dir) {
    constexpr int P = Ring<A>::P;
    constexpr int U = Ring<A>::U;
    const int lane = threadIdx.x;
    const int j0 = cs + lane * V;
    bool col_in[V];
#pragma unroll
    for (int e = 0; e < V; ++e) col_in[e] = (j0 + e >= 1) && (j0 + e <= W - 2);
    // store offsets (bytes within the row): the lane's columns inside [olo, ohi), else dropped
    const bool st_lane = (j0 >= olo) && (j0 + V <= ohi);
    const uint32_t voff_vec = st_lane ? (uint32_t)j0 * (uint32_t)sizeof(T) : kDropOffset;
    uint32_t voff_el[V];
#pragma unroll
    for (int e = 0; e < V; ++e)
        voff_el[e] = (j0 + e >= olo && j0 + e < ohi && col_in[e]) ? (uint32_t)(j0 + e) * (uint32_t)sizeof(T)
                                                                   : kDropOffset;

    // step t loads row L0 + dir*t; the band's rows [rb, re) are stored
    const int L0 = dir > 0 ? rb - TL : re - 1 + TL;
    const int nsteps = (re - rb) + 2 * TL;
    __builtin_amdgcn_s_setprio(3);
    T w0[TL][V], w1[TL][V];
    T ring[P][V];
#pragma unroll
    for (int i = 0; i < A; ++i) stream_load<T, V, EDGE>(in, L0 + dir * i, H, W, ld, j0, ring[i]);
    stream_prologue<T, V, TL, A, 0, EDGE>(w0, w1, ring, in, L0, dir, H, W, ld, j0, c, col_in);

    // Groups of U steps; level rows of step t are L - dir*s for s = 1..TL and
    // leave [1, H-2] only where the loaded row is outside the grid. The last
    // group may run past the band (at most U-1 steps): those steps compute
    // rows that are not stored (and loads stay clamped to the grid).
    const int ngroups = (nsteps - 2 * TL + U - 1) / U;
    int quarter = 0;
    for (int k = 0; k < ngroups; ++k) {
        const int q = (4 * k) / ngroups;
        if (q != quarter) {
            quarter = q;
            if (q == 1)
                __builtin_amdgcn_s_setprio(2);
            else if (q == 2)
                __builtin_amdgcn_s_setprio(1);
            else
                __builtin_amdgcn_s_setprio(0);
        }
        const int g = 2 * TL + k * U;
        const int La = L0 + dir * g, Lb = L0 + dir * (g + U - 1);
        const bool rowchk = min(La, Lb) < 0 || max(La, Lb) > H - 1;
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int t = 2 * TL + i;  // step index modulo U (g - 2*TL is a multiple of U)
            const int L = L0 + dir * (g + i);
            T top[V];
            if (!rowchk)
                stream_step<T, V, TL, TL, EDGE, false>(w0, w1, ring[(t + P - 2) % P], ring[(t + P - 1) % P],
                                                       ring[t % P], top, L, dir, H, c, col_in);
            else
                stream_step<T, V, TL, TL, EDGE, true>(w0, w1, ring[(t + P - 2) % P], ring[(t + P - 1) % P],
                                                      ring[t % P], top, L, dir, H, c, col_in);
            stream_load<T, V, EDGE>(in, L + dir * A, H, W, ld, j0, ring[(t + A) % P]);
            stream_store<T, V, EDGE>(out, L - dir * TL, ld, W, g + i < nsteps, voff_vec, voff_el, top);
            // keep steps apart: interleaving them only hoists lane shifts and
            // loads, which costs registers (occupancy) and gains nothing
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Strip layout. Flush layout (flush != 0: W is a multiple of V and at least
// 64*V): strip 0 loads columns [0, 64V) and stores [0, 64V - HALO); strip k
// loads from k*OW and stores [k*OW + HALO, (k+1)*OW + HALO); the last strip
// loads the grid's last 64V columns and stores [W - 64V + HALO, W). Only the
// first and last strips touch a boundary column, and all loads stay inside the
// grid. The last strip's stores may overlap its neighbour's: both compute the
// same bits there. Otherwise (flush == 0) strip k loads from k*OW - HALO and
// stores [k*OW, (k+1)*OW); the first and last strips load past the grid.
// Workgroup `tile` of a grid walks band tile / strips of strip tile % strips.
template <typename T, int V, int TL, int A>
__device__ __forceinline__ void stream_tile(const T* __restrict__ in, T* __restrict__ out, int H, int W, int64_t ld,
                                            T c, uint32_t strips, int band, int flush, uint32_t tile) {
    constexpr int HALO = (TL + V - 1) / V * V;
    constexpr int OW = 64 * V - 2 * HALO;
    const uint32_t bi = tile / strips;
    const uint32_t strip = tile - bi * strips;
    int cs, olo, ohi;  // first loaded column (a multiple of V), stored columns [olo, ohi)
    if (flush) {
        const bool last = strip == strips - 1;
        cs = last ? W - 64 * V : (int)strip * OW;
        olo = strip == 0 ? 0 : cs + HALO;
        ohi = last ? W : cs + HALO + OW;
    } else {
        cs = (int)strip * OW - HALO;
        olo = cs + HALO;
        ohi = olo + OW;
    }
    const int rb = 1 + (int)bi * band;
    const int re = min(rb + band, H - 1);
    const int dir = (bi & 1) ? -1 : 1;
    if (cs >= 1 && cs + 64 * V <= W - 1)
        stream_band<T, V, TL, A, 0>(in, out, H, W, ld, c, cs, olo, ohi, rb, re, dir);
    else if (flush)
        stream_band<T, V, TL, A, 1>(in, out, H, W, ld, c, cs, olo, ohi, rb, re, dir);
    else
        stream_band<T, V, TL, A, 2>(in, out, H, W, ld, c, cs, olo, ohi, rb, re, dir);
}

// FP64: keep 3 waves per SIMD (at most 168 VGPRs). The 12-level kernel needs
// 169 otherwise and would drop to 2; under the cap it spills one 8-byte value,
// stored once per wave and reloaded once per band, outside the row loop.
#define STEN_STREAM_OCCUPANCY __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 1)))

template <typename T, int V, int TL, int A>
__global__ __launch_bounds__(64) STEN_STREAM_OCCUPANCY void sweep_stream_kernel(const T* __restrict__ in, T* __restrict__ out, int H, int W,
                                                         int64_t ld, T c, uint32_t strips, int band, int flush) {
    stream_tile<T, V, TL, A>(in, out, H, W, ld, c, strips, band, flush, xcd_tile_of_block(blockIdx.x, gridDim.x));
}

// Several grids in one launch: grid k owns the workgroups [first, first +
// strips * bands) of the launch, numbered after the XCD-aware map, and runs
// them as the one-grid kernel would. Grids are independent (no aliasing).
template <typename T>
struct StreamGrid {
    const T* in;
    T* out;
    int64_t ld;
    int H, W;
    uint32_t strips, first;
    int band, flush;
};

constexpr int kMaxStreamGrids = kMaxStreamGridsPerLaunch;

template <typename T>
struct StreamGrids {
    StreamGrid<T> g[kMaxStreamGrids];
    int n;
};

template <typename T, int V, int TL, int A>
__global__ __launch_bounds__(64) STEN_STREAM_OCCUPANCY void sweep_stream_grids_kernel(const StreamGrids<T> grids, T c) {
    const uint32_t b = xcd_tile_of_block(blockIdx.x, gridDim.x);
    int k = 0;
    while (k + 1 < grids.n && b >= grids.g[k + 1].first) ++k;
    const StreamGrid<T>& g = grids.g[k];
    stream_tile<T, V, TL, A>(g.in, g.out, g.H, g.W, g.ld, c, g.strips, g.band, g.flush, b - g.first);
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

// Process-wide tuning settings. Each is read atomically wherever a launch is
// configured, and every value a setter accepts gives the same results, so a
// call racing a setter runs some valid mix of old and new settings.
std::atomic<int> g_tb_rows{0};     // output rows per register tile (0: 8)
std::atomic<int> g_tb_variant{0};  // 0: built-in (streaming), 1: register tile where it has the level count, 2: streaming
std::atomic<int> g_tb_band{0};     // streaming: output rows per band (0: built-in)
std::atomic<int> g_tb_depth{0};    // streaming: rows loaded ahead (0 or 4; loading 7 ahead measured no faster)

constexpr int kStreamDepth = 4;
constexpr int kMaxBlockLevels = 6;
constexpr int kMaxStreamLevels = 12;

// false (nothing launched) for a level count without a kernel
template <typename T, int V, int ROWS>
bool launch_levels_rows(const T* in, T* out, int H, int W, int64_t ld, T c, int levels, hipStream_t s) {
    switch (levels) {
        case 1: launch_tb<T, V, ROWS, 1>(in, out, H, W, ld, c, s); return true;
        case 2: launch_tb<T, V, ROWS, 2>(in, out, H, W, ld, c, s); return true;
        case 3: launch_tb<T, V, ROWS, 3>(in, out, H, W, ld, c, s); return true;
        case 4: launch_tb<T, V, ROWS, 4>(in, out, H, W, ld, c, s); return true;
        case 5: launch_tb<T, V, ROWS, 5>(in, out, H, W, ld, c, s); return true;
        case 6: launch_tb<T, V, ROWS, 6>(in, out, H, W, ld, c, s); return true;
        default: return false;
    }
}

// One register-tile launch of `levels` sweeps (1..6).
template <typename T, int V>
bool launch_levels_block(const T* in, T* out, int H, int W, int64_t ld, T c, int levels, hipStream_t s) {
    switch (g_tb_rows.load(std::memory_order_relaxed)) {
        case 4: return launch_levels_rows<T, V, 4>(in, out, H, W, ld, c, levels, s);
        case 12: return launch_levels_rows<T, V, 12>(in, out, H, W, ld, c, levels, s);
        case 16: return launch_levels_rows<T, V, 16>(in, out, H, W, ld, c, levels, s);
        default: return launch_levels_rows<T, V, 8>(in, out, H, W, ld, c, levels, s);
    }
}

// Waves of one kernel that fit on the device at once (one wave per workgroup).
int resident_waves(const void* kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess)
        return 0;
    return cus * per_cu;
}

template <typename T, int V, int TL, int D>
void launch_stream(const T* in, T* out, int H, int W, int64_t ld, T c, hipStream_t s) {
    constexpr int HALO = (TL + V - 1) / V * V;
    constexpr int OW = 64 * V - 2 * HALO;
    const int flush = (W % V == 0 && W >= 64 * V) ? 1 : 0;
    // flush: enough regular strips that the last (right-aligned) strip meets them; else strip k
    // stores columns [k*OW, (k+1)*OW)
    const uint32_t strips = flush ? ceil_div(W - 64 * V, OW) + 1 : ceil_div(W - 1, OW);
    int band = g_tb_band.load(std::memory_order_relaxed);
    if (band <= 0) {
        // Built-in: the tallest bands that still give every resident wave slot
        // a band, so the grid runs in one round; at least 2*TL rows, so a band
        // start (2*TL steps) costs at most as much as the band itself.
        static const int waves = resident_waves(reinterpret_cast<const void*>(&sweep_stream_kernel<T, V, TL, D>));
        const int64_t fit = std::max<int64_t>(1, (waves > 0 ? waves : 1024) / (int64_t)strips);
        band = (int)std::max<int64_t>(2 * TL, (H - 2 + fit - 1) / fit);
    }
    const uint32_t bands = ceil_div(H - 2, band);
    sweep_stream_kernel<T, V, TL, D><<<strips * bands, 64, 0, s>>>(in, out, H, W, ld, c, strips, band, flush);
}

// FP64 launches of 13 or 14 sweeps: the streaming kernel's code at 2 waves
// per SIMD (its 190-200 VGPRs do not fit 3). Where HBM serves the grid, the
// deeper pass is faster per sweep than 12 levels at 3 waves; at 4096^2, where
// the pair of buffers sits in the Infinity Cache, it is not.
template <int TL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void sweep_stream_deep_kernel(
    const double* __restrict__ in, double* __restrict__ out, int H, int W, int64_t ld, double c, uint32_t strips,
    int band, int flush) {
    stream_tile<double, 2, TL, kStreamDepth>(in, out, H, W, ld, c, strips, band, flush,
                                             xcd_tile_of_block(blockIdx.x, gridDim.x));
}

template <int TL>
void launch_stream_deep(const double* in, double* out, int H, int W, int64_t ld, double c, hipStream_t s) {
    constexpr int V = 2;
    constexpr int HALO = (TL + V - 1) / V * V;
    constexpr int OW = 64 * V - 2 * HALO;
    const int flush = (W % V == 0 && W >= 64 * V) ? 1 : 0;
    const uint32_t strips = flush ? ceil_div(W - 64 * V, OW) + 1 : ceil_div(W - 1, OW);
    int band = g_tb_band.load(std::memory_order_relaxed);
    if (band <= 0) {
        static const int waves = resident_waves(reinterpret_cast<const void*>(&sweep_stream_deep_kernel<TL>));
        const int64_t fit = std::max<int64_t>(1, (waves > 0 ? waves : 1024) / (int64_t)strips);
        band = (int)std::max<int64_t>(2 * TL, (H - 2 + fit - 1) / fit);
    }
    const uint32_t bands = ceil_div(H - 2, band);
    sweep_stream_deep_kernel<TL><<<strips * bands, 64, 0, s>>>(in, out, H, W, ld, c, strips, band, flush);
}

template <typename T, int V, int D>
bool launch_stream_depth(const T* in, T* out, int H, int W, int64_t ld, T c, int levels, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (levels == 13) {
            launch_stream_deep<13>(in, out, H, W, ld, c, s);
            return true;
        }
        if (levels == 14) {
            launch_stream_deep<14>(in, out, H, W, ld, c, s);
            return true;
        }
    }
    switch (levels) {
        case 1: launch_stream<T, V, 1, D>(in, out, H, W, ld, c, s); return true;
        case 2: launch_stream<T, V, 2, D>(in, out, H, W, ld, c, s); return true;
        case 3: launch_stream<T, V, 3, D>(in, out, H, W, ld, c, s); return true;
        case 4: launch_stream<T, V, 4, D>(in, out, H, W, ld, c, s); return true;
        case 5: launch_stream<T, V, 5, D>(in, out, H, W, ld, c, s); return true;
        case 6: launch_stream<T, V, 6, D>(in, out, H, W, ld, c, s); return true;
        case 7: launch_stream<T, V, 7, D>(in, out, H, W, ld, c, s); return true;
        case 8: launch_stream<T, V, 8, D>(in, out, H, W, ld, c, s); return true;
        case 9: launch_stream<T, V, 9, D>(in, out, H, W, ld, c, s); return true;
        case 10: launch_stream<T, V, 10, D>(in, out, H, W, ld, c, s); return true;
        case 11: launch_stream<T, V, 11, D>(in, out, H, W, ld, c, s); return true;
        case 12: launch_stream<T, V, 12, D>(in, out, H, W, ld, c, s); return true;
        default: return false;
    }
}

// One launch of TL sweeps on each of n independent grids (n <= kMaxStreamGrids).
// Band heights follow the one-grid rule with the strips of all grids together,
// so the whole launch fits the device's resident wave slots in one round.
template <typename T, int V, int TL, int D>
void launch_stream_grids(const GridView<T>* views, int n, T c, hipStream_t s) {
    constexpr int HALO = (TL + V - 1) / V * V;
    constexpr int OW = 64 * V - 2 * HALO;
    StreamGrids<T> args{};
    args.n = n;
    int64_t all_strips = 0;
    for (int k = 0; k < n; ++k) {
        StreamGrid<T>& g = args.g[k];
        g.in = views[k].in;
        g.out = views[k].out;
        g.ld = views[k].ld;
        g.H = views[k].H;
        g.W = views[k].W;
        g.flush = (g.W % V == 0 && g.W >= 64 * V) ? 1 : 0;
        g.strips = g.flush ? ceil_div(g.W - 64 * V, OW) + 1 : ceil_div(g.W - 1, OW);
        all_strips += g.strips;
    }
    static const int waves =
        resident_waves(reinterpret_cast<const void*>(&sweep_stream_grids_kernel<T, V, TL, D>));
    const int64_t fit = std::max<int64_t>(1, (waves > 0 ? waves : 1024) / std::max<int64_t>(1, all_strips));
    uint32_t first = 0;
    const int band_set = g_tb_band.load(std::memory_order_relaxed);
    for (int k = 0; k < n; ++k) {
        StreamGrid<T>& g = args.g[k];
        g.band = band_set > 0 ? band_set : (int)std::max<int64_t>(2 * TL, (g.H - 2 + fit - 1) / fit);
        g.first = first;
        first += g.strips * ceil_div(g.H - 2, g.band);
    }
    if (first > 0) sweep_stream_grids_kernel<T, V, TL, D><<<first, 64, 0, s>>>(args, c);
}

template <typename T, int V, int D>
bool launch_stream_grids_depth(const GridView<T>* views, int n, T c, int levels, hipStream_t s) {
    switch (levels) {
        case 1: launch_stream_grids<T, V, 1, D>(views, n, c, s); return true;
        case 2: launch_stream_grids<T, V, 2, D>(views, n, c, s); return true;
        case 3: launch_stream_grids<T, V, 3, D>(views, n, c, s); return true;
        case 4: launch_stream_grids<T, V, 4, D>(views, n, c, s); return true;
        case 5: launch_stream_grids<T, V, 5, D>(views, n, c, s); return true;
        case 6: launch_stream_grids<T, V, 6, D>(views, n, c, s); return true;
        case 7: launch_stream_grids<T, V, 7, D>(views, n, c, s); return true;
        case 8: launch_stream_grids<T, V, 8, D>(views, n, c, s); return true;
        case 9: launch_stream_grids<T, V, 9, D>(views, n, c, s); return true;
        case 10: launch_stream_grids<T, V, 10, D>(views, n, c, s); return true;
        case 11: launch_stream_grids<T, V, 11, D>(views, n, c, s); return true;
        case 12: launch_stream_grids<T, V, 12, D>(views, n, c, s); return true;
        default: return false;
    }
}

// One blocked launch of `levels` sweeps (1..12; FP64 1..14). The register tile has 1..6
// levels: it runs when asked for (variant 1) or when rows are too wide for
// the streaming kernel, and only for a level count it has. Returns false, with
// nothing launched, for a level count no kernel has (wide rows: above 6).
template <typename T, int V>
bool launch_levels(const T* in, T* out, int H, int W, int64_t ld, T c, int levels, hipStream_t s) {
    // the streaming kernel addresses a row with 32-bit byte offsets
    const bool stream_fits = (int64_t)W * (int64_t)sizeof(T) < ((int64_t)1 << 30);
    if (levels <= kMaxBlockLevels && (!stream_fits || g_tb_variant.load(std::memory_order_relaxed) == 1))
        return launch_levels_block<T, V>(in, out, H, W, ld, c, levels, s);
    if (!stream_fits) return false;
    return launch_stream_depth<T, V, kStreamDepth>(in, out, H, W, ld, c, levels, s);
}

template <typename T>
sten_status run_tb(const T* u0, T* out, T* work, int64_t H, int64_t W, int64_t ld, int32_t T_, T c, int32_t tl,
                   hipStream_t stream) {
    if (tl < 1 || tl > max_stream_levels<T>()) return STEN_ERR_ARG;
    // rows too wide for the streaming kernel's 32-bit offsets take the register tile
    if (W * (int64_t)sizeof(T) >= ((int64_t)1 << 30)) tl = std::min(tl, kMaxBlockLevels);
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
    // launch k (1-based) applies `lev` sweeps, the T sweeps split as evenly as the
    // launch count allows (each at most tl); the last launch must write `out`
    const T* src = u0;
    const int base = T_ / launches, extra = T_ % launches;
    for (int k = 1; k <= launches; ++k) {
        const int lev = base + (k <= extra ? 1 : 0);
        T* dst = ((launches - k) % 2 == 0) ? out : work;
        if (!launch_levels<T, VV>(src, dst, h, w, ld, c, lev, stream)) return STEN_ERR_ARG;  // unreachable: lev <= tl
        src = dst;
    }
    return check_launch();
}

}  // namespace

// `levels` sweeps (1..12) on each of n independent grids, in launches of up to
// kMaxStreamGrids grids. Each grid: H, W >= 3, in and out 16-byte aligned, ld
// even and W * 8 below 2^30 bytes; the caller checks these.
// Returns false, with nothing launched, for levels outside 1..12.
bool launch_stream_grids_f64(const GridView<double>* views, int n, double c, int levels, hipStream_t s) {
    if (levels < 1 || levels > kMaxStreamLevels) return false;
    for (int k = 0; k < n; k += kMaxStreamGrids)
        launch_stream_grids_depth<double, 2, kStreamDepth>(views + k, std::min(n - k, kMaxStreamGrids), c, levels,
                                                           s);
    return true;
}

// One blocked launch of `levels` sweeps (1..14) from in to out, FP64 (no
// argument checks; 16-byte aligned data, even ld). Returns false, with
// nothing launched, for a level count no kernel has.
bool launch_levels_f64(const double* in, double* out, int H, int W, int64_t ld, double c, int levels,
                       hipStream_t s) {
    return launch_levels<double, 2>(in, out, H, W, ld, c, levels, s);
}

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

sten_status sten_tune_tb(int32_t variant, int32_t band, int32_t depth) {
    if (variant < 0 || variant > 2 || band < 0 || band > 65536) return STEN_ERR_ARG;
    if (depth != 0 && depth != sten::kStreamDepth) return STEN_ERR_ARG;
    sten::g_tb_variant = variant;
    sten::g_tb_band = band;
    sten::g_tb_depth = depth;
    return STEN_OK;
}

sten_status sten_tune_tb_rows(int32_t rows) {
    if (rows != 0 && rows != 4 && rows != 8 && rows != 12 && rows != 16) return STEN_ERR_ARG;
    sten::g_tb_rows = rows;
    return STEN_OK;
}

}  // extern "C"
