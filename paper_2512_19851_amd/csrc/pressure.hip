// Temporal blocking of the lid-driven cavity flow's pressure iteration (the
// paper's second benchmark, Section V): several Jacobi iterations of the
// pressure equation, each with its wall conditions, per pass over HBM, with
// the same bits as running them one at a time.
//
// One iteration maps p to q (b is the source term, fixed during the solve):
//   q[i,j] = (cw * (p[i,j+1] + p[i,j-1]) + cn * (p[i+1,j] + p[i-1,j])) - cb * b[i,j]
//            on the interior rows 1..H-2 and columns 1..W-2;
//   q[i,W-1] = q[i,W-2] and q[i,0] = q[i,1] on rows 1..H-2   (dp/dx = 0, side walls);
//   q[0,:] = q[1,:]                                           (dp/dy = 0, bottom wall, corners included);
//   q[H-1,:] = 0                                              (p = 0 on the lid).
//
// The walk is the streaming blocked kernel's: a wave owns a strip of 64 lanes
// x 2 FP64 columns and walks a band of rows; level s of row r comes from level
// s-1 of rows r-1, r, r+1, kept in registers. Three things are added:
//  * b: each level reads b at its own row. b rows are loaded with the p rows
//    (same step, same clamped row) into a ring long enough that the deepest
//    level still finds its row: level s reads, at step t, the b row loaded for
//    step t - s, and a slot is reloaded only PB >= TL + A steps later (up to 8
//    levels; deeper passes keep the ring in LDS, below).
//  * side walls: only the grid-aligned strip layout is used (W even, W >= 128),
//    so column 0 and column 1 sit in lane 0 of the first strip and columns
//    W-2, W-1 in lane 63 of the last: the copies are lane-local selects.
//  * bottom wall and lid: as a level passes row H-1 it becomes 0; row 0 of a
//    level is row 1 of that level. Walking down, row 0 is produced before
//    row 1, so when row 1 appears it overwrites the kept row-0 value before the
//    next level reads it; walking up, row 0 takes the kept row-1 value. The
//    last level keeps no rows: the band that stores row 1 also stores it as
//    row 0, and no band stores row H-1 (the output's lid row is zeroed once).
// Every stored value is the one-iteration-at-a-time value: each point of each
// level is the same expression on the same operands, evaluated in the same
// order, without contraction. b does not change during the solve, so the
// product cb * b[i,j] is formed once per row and pass, as the row is staged:
// the same rounded value every iteration would form.
//
// Passes of more than 8 levels keep the b rows in LDS instead (the register
// ring no longer fits beside the levels' rows): each b row is loaded into a
// short register staging ring, written to a per-wave LDS ring of R >= TL rows
// once it has arrived, and read back once per level.
#include <algorithm>
#include <atomic>

#include "common.hpp"
#include "stream_common.hpp"

namespace sten {
namespace {

using namespace stream;

constexpr int kPV = 2;  // FP64 values per lane
constexpr int kPA = 4;  // rows loaded ahead

// BEGIN KERNEL SOURCE (the HBM traffic measurement is keyed to this region)
typedef TVec<double, kPV>::type PVec;

// LB false: b rows in a register ring of PB >= TL + A slots. LB true: b rows
// staged in PB = P register slots, then kept in an LDS ring of R >= TL rows.
template <int TL, bool LB>
struct PressureRing {
    static constexpr int P = kPA + 2;                             // p rows: step t reads the rows of steps t-2..t
    static constexpr int PB = LB ? P : (TL + kPA + 5) / 6 * 6;    // b rows in registers (a multiple of 6)
    static constexpr int R = LB ? (TL + 5) / 6 * 6 : 0;           // b rows in LDS: a multiple of 6 and >= TL
    static constexpr int U = LB ? R : PB;                         // group length: a multiple of P, PB and R
};

// The scaled b row (cb * b) of step u for one level: from the register ring,
// or from LDS (row u of the wave's LDS ring; 64 lanes x 16 bytes per row).
template <int TL, bool LB>
__device__ __forceinline__ void level_b(const double (&bring)[PressureRing<TL, LB>::PB][kPV],
                                        const PVec* __restrict__ lb, int u, double (&bb)[kPV]) {
    if constexpr (LB) {
        const PVec v = lb[(u % PressureRing<TL, LB>::R) * 64 + (int)threadIdx.x];
        bb[0] = v[0];
        bb[1] = v[1];
    } else {
#pragma unroll
        for (int e = 0; e < kPV; ++e) bb[e] = bring[u % PressureRing<TL, LB>::PB][e];
    }
}

// After step u, the b row of step u has arrived: it is scaled by cb, in place
// in the register ring, or on its way to LDS row u. Levels read it from step
// u + 1 on; with R >= TL the LDS row it replaces, step u - R, was last read by
// level TL at step u - R + TL <= u.
template <int TL, bool LB, typename RG = PressureRing<TL, LB>>
__device__ __forceinline__ void stage_b(double (&bring)[RG::PB][kPV], PVec* __restrict__ lb, int u, double cb) {
    constexpr int PB = RG::PB;
    if constexpr (LB) {
        PVec v;
        v[0] = cb * bring[u % PB][0];
        v[1] = cb * bring[u % PB][1];
        lb[(u % RG::R) * 64 + (int)threadIdx.x] = v;
    } else {
#pragma unroll
        for (int e = 0; e < kPV; ++e) bring[u % PB][e] = cb * bring[u % PB][e];
    }
}

// One level of one row from the level below: a and c are its vertical
// neighbours (in either order), m the row itself, sb the scaled source term
// cb * b. fix_lo / fix_hi: this lane holds column 0 / column W-1 (side-wall
// copies).
template <bool EDGE>
__device__ __forceinline__ void pressure_level(const double (&a)[kPV], const double (&m)[kPV], const double (&c)[kPV],
                                               const double (&sb)[kPV], double (&res)[kPV], double cw, double cn,
                                               bool fix_lo, bool fix_hi) {
    const double lft = lane_from_lower(m[1]);  // column j0 - 1
    const double rgt = lane_from_upper(m[0]);  // column j0 + 2
    const double h0 = m[1] + lft;              // east + west of column j0
    const double h1 = rgt + m[0];              // east + west of column j0 + 1
    const double v0 = (cw * h0 + cn * (c[0] + a[0])) - sb[0];
    const double v1 = (cw * h1 + cn * (c[1] + a[1])) - sb[1];
    res[0] = (EDGE && fix_lo) ? v1 : v0;
    res[1] = (EDGE && fix_hi) ? v0 : v1;
}

// Bottom wall and lid for level s's row r (cur); prev is the row this level
// produced one step earlier (absent for the last level). Written as bit masks
// on the FP64 patterns (the lid value is +0.0, all bits clear): as plain
// selects on wave-uniform conditions the compiler emits branches inside the
// unrolled steps, which cost registers.
template <bool HAS_PREV>
__device__ __forceinline__ void pressure_rows(double (&cur)[kPV], double (&prev)[kPV], int r, int dir, int H) {
    const uint64_t keep = r == H - 1 ? 0ull : ~0ull;
    const uint64_t take = (HAS_PREV && dir < 0 && r == 0) ? ~0ull : 0ull;
    const uint64_t give = (HAS_PREV && dir > 0 && r == 1) ? ~0ull : 0ull;
#pragma unroll
    for (int e = 0; e < kPV; ++e) {
        const uint64_t c = __builtin_bit_cast(uint64_t, cur[e]);
        const uint64_t q = __builtin_bit_cast(uint64_t, prev[e]);
        const uint64_t v = ((q & take) | (c & ~take)) & keep;
        if constexpr (HAS_PREV) prev[e] = __builtin_bit_cast(double, (v & give) | (q & ~give));
        cur[e] = __builtin_bit_cast(double, v);
    }
}

// One step: the level-0 row L (x) enters; levels 1..NACT advance by one row
// each (level s produces row L - dir*s from the level below and the b row
// loaded for step t - s; t is a constant once the caller's loop is unrolled).
// w0[k], w1[k] hold the two latest rows of level k >= 1, older first. With
// NACT == TL the level-TL row goes to `top`.
template <int TL, int NACT, bool EDGE, bool ROWCHK, bool LB>
__device__ __forceinline__ void pressure_step(double (&w0)[TL][kPV], double (&w1)[TL][kPV], const double (&a0)[kPV],
                                              const double (&b0)[kPV], const double (&x)[kPV],
                                              const double (&bring)[PressureRing<TL, LB>::PB][kPV],
                                              const PVec* __restrict__ lb, double (&top)[kPV], int t, int L, int dir,
                                              int H, double cw, double cn, bool fix_lo, bool fix_hi) {
    if constexpr (NACT >= 1) {
        double cur[kPV];
        double b1[kPV];
        level_b<TL, LB>(bring, lb, t - 1, b1);
        pressure_level<EDGE>(a0, b0, x, b1, cur, cw, cn, fix_lo, fix_hi);
        if constexpr (ROWCHK) pressure_rows<(1 < TL)>(cur, w1[1 < TL ? 1 : 0], L - dir, dir, H);
#pragma unroll
        for (int s = 2; s <= NACT; ++s) {
            double nv[kPV];
            double bs[kPV];
            level_b<TL, LB>(bring, lb, t - s, bs);
            pressure_level<EDGE>(w0[s - 1], w1[s - 1], cur, bs, nv, cw, cn, fix_lo, fix_hi);
#pragma unroll
            for (int e = 0; e < kPV; ++e) {
                w0[s - 1][e] = w1[s - 1][e];
                w1[s - 1][e] = cur[e];
                cur[e] = nv[e];
            }
            if constexpr (ROWCHK) {
                if (s < TL)
                    pressure_rows<true>(cur, w1[s < TL ? s : 0], L - dir * s, dir, H);
                else
                    pressure_rows<false>(cur, w1[0], L - dir * s, dir, H);
            }
        }
        if constexpr (NACT < TL) {
#pragma unroll
            for (int e = 0; e < kPV; ++e) {
                w0[NACT][e] = w1[NACT][e];
                w1[NACT][e] = cur[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < kPV; ++e) top[e] = cur[e];
        }
    }
}

// Steps 0 .. 2*TL-1: level s is complete from step 2s on.
template <int TL, int K, bool EDGE, bool LB, typename RG = PressureRing<TL, LB>>
__device__ __forceinline__ void pressure_prologue(double (&w0)[TL][kPV], double (&w1)[TL][kPV],
                                                  double (&ring)[RG::P][kPV], double (&bring)[RG::PB][kPV],
                                                  PVec* __restrict__ lb, const double* __restrict__ p,
                                                  const double* __restrict__ b, int L0, int dir, int H, int W,
                                                  int64_t ld, int j0, double cw, double cn, double cb, bool fix_lo,
                                                  bool fix_hi) {
    constexpr int P = RG::P;
    constexpr int PB = RG::PB;
    if constexpr (K < 2 * TL) {
        double unused[kPV];
        pressure_step<TL, K / 2, EDGE, true, LB>(w0, w1, ring[(K + P - 2) % P], ring[(K + P - 1) % P],
                                                 ring[K % P], bring, lb, unused, K, L0 + dir * K, dir, H, cw, cn,
                                                 fix_lo, fix_hi);
        stage_b<TL, LB>(bring, lb, K, cb);
        stream_load<double, kPV, 1>(p, L0 + dir * (K + kPA), H, W, ld, j0, ring[(K + kPA) % P]);
        stream_load<double, kPV, 1>(b, L0 + dir * (K + kPA), H, W, ld, j0, bring[(K + kPA) % PB]);
        __builtin_amdgcn_sched_barrier(0);
        pressure_prologue<TL, K + 1, EDGE, LB>(w0, w1, ring, bring, lb, p, b, L0, dir, H, W, ld, j0, cw, cn, cb,
                                               fix_lo, fix_hi);
    }
}

template <int TL, bool EDGE, bool LB>
__device__ __forceinline__ void pressure_band(const double* __restrict__ p, const double* __restrict__ b,
                                              double* __restrict__ out, PVec* __restrict__ lb, int H, int W,
                                              int64_t ld, double cw, double cn, double cb, int cs, int olo, int ohi,
                                              int rb, int re, int dir) {
    constexpr int P = PressureRing<TL, LB>::P;
    constexpr int PB = PressureRing<TL, LB>::PB;
    constexpr int U = PressureRing<TL, LB>::U;
    const int lane = threadIdx.x;
    const int j0 = cs + lane * kPV;
    const bool fix_lo = j0 == 0;
    const bool fix_hi = j0 + 1 == W - 1;
    const bool st_lane = (j0 >= olo) && (j0 + kPV <= ohi);
    const uint32_t voff_vec = st_lane ? (uint32_t)j0 * (uint32_t)sizeof(double) : kDropOffset;
    const uint32_t voff_el[kPV] = {kDropOffset, kDropOffset};  // unused by whole-vector stores

    const int L0 = dir > 0 ? rb - TL : re - 1 + TL;
    const int nsteps = (re - rb) + 2 * TL;
    __builtin_amdgcn_s_setprio(3);
    double w0[TL][kPV], w1[TL][kPV];
    double ring[P][kPV];
    double bring[PB][kPV];
#pragma unroll
    for (int i = 0; i < kPA; ++i) {
        stream_load<double, kPV, 1>(p, L0 + dir * i, H, W, ld, j0, ring[i]);
        stream_load<double, kPV, 1>(b, L0 + dir * i, H, W, ld, j0, bring[i]);
    }
    pressure_prologue<TL, 0, EDGE, LB>(w0, w1, ring, bring, lb, p, b, L0, dir, H, W, ld, j0, cw, cn, cb, fix_lo,
                                       fix_hi);

    // Groups of U steps. The bottom and lid rows need per-row handling only in
    // groups whose level rows come within TL rows of them; the last group may
    // run past the band (steps computed, not stored). One loop body with the
    // per-row variant chosen per step keeps one register assignment for the
    // rings across the loop.
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
        const bool rowchk = min(La, Lb) - TL <= 1 || max(La, Lb) + TL >= H - 1;
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int t = 2 * TL + i;  // step index modulo U (g - 2*TL is a multiple of U)
            const int L = L0 + dir * (g + i);
            const int r = L - dir * TL;
            const bool live = g + i < nsteps;
            double top[kPV];
            if (!rowchk) {
                pressure_step<TL, TL, EDGE, false, LB>(w0, w1, ring[(t + P - 2) % P], ring[(t + P - 1) % P],
                                                       ring[t % P], bring, lb, top, t, L, dir, H, cw, cn, fix_lo,
                                                       fix_hi);
            } else {
                pressure_step<TL, TL, EDGE, true, LB>(w0, w1, ring[(t + P - 2) % P], ring[(t + P - 1) % P],
                                                      ring[t % P], bring, lb, top, t, L, dir, H, cw, cn, fix_lo,
                                                      fix_hi);
                // the bottom wall: row 0 of the last level is its row 1
                stream_store<double, kPV, 1>(out, 0, ld, W, live && r == 1, voff_vec, voff_el, top);
            }
            stage_b<TL, LB>(bring, lb, t, cb);
            stream_load<double, kPV, 1>(p, L + dir * kPA, H, W, ld, j0, ring[(t + kPA) % P]);
            stream_load<double, kPV, 1>(b, L + dir * kPA, H, W, ld, j0, bring[(t + kPA) % PB]);
            stream_store<double, kPV, 1>(out, r, ld, W, live, voff_vec, voff_el, top);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Grid-aligned strip layout (W even, W >= 128): strip 0 loads columns
// [0, 128) and stores [0, 128 - HALO); strip k loads from k*OW and stores
// [k*OW + HALO, (k+1)*OW + HALO); the last strip loads the last 128 columns
// and stores [W - 128 + HALO, W). All loads stay inside the grid; the last
// strip's stores may overlap its neighbour's with the same bits.
template <int TL, bool LB>
__device__ __forceinline__ void pressure_tile(const double* __restrict__ p, const double* __restrict__ b,
                                              double* __restrict__ out, PVec* __restrict__ lb, int H, int W,
                                              int64_t ld, double cw, double cn, double cb, uint32_t strips,
                                              int band) {
    constexpr int HALO = (TL + kPV - 1) / kPV * kPV;
    constexpr int OW = 64 * kPV - 2 * HALO;
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t bi = tile / strips;
    const uint32_t strip = tile - bi * strips;
    const bool last = strip == strips - 1;
    const int cs = last ? W - 64 * kPV : (int)strip * OW;
    const int olo = strip == 0 ? 0 : cs + HALO;
    const int ohi = last ? W : cs + HALO + OW;
    const int rb = 1 + (int)bi * band;
    const int re = min(rb + band, H - 1);
    const int dir = (bi & 1) ? -1 : 1;
    if (strip == 0 || last)
        pressure_band<TL, true, LB>(p, b, out, lb, H, W, ld, cw, cn, cb, cs, olo, ohi, rb, re, dir);
    else
        pressure_band<TL, false, LB>(p, b, out, lb, H, W, ld, cw, cn, cb, cs, olo, ohi, rb, re, dir);
}

// Up to 8 levels: b rows in registers.
template <int TL>
__global__ __launch_bounds__(64) void pressure_stream_kernel(const double* __restrict__ p,
                                                             const double* __restrict__ b, double* __restrict__ out,
                                                             int H, int W, int64_t ld, double cw, double cn, double cb,
                                                             uint32_t strips, int band) {
    pressure_tile<TL, false>(p, b, out, nullptr, H, W, ld, cw, cn, cb, strips, band);
}

// 9 to 12 levels: b rows in a per-wave LDS ring (R KiB per one-wave workgroup),
// 2 waves per SIMD.
template <int TL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void pressure_stream_lds_kernel(
    const double* __restrict__ p, const double* __restrict__ b, double* __restrict__ out, int H, int W, int64_t ld,
    double cw, double cn, double cb, uint32_t strips, int band) {
    __shared__ PVec lb[PressureRing<TL, true>::R * 64];
    pressure_tile<TL, true>(p, b, out, lb, H, W, ld, cw, cn, cb, strips, band);
}
// END KERNEL SOURCE

// Row H-1 of one or two grids := 0 (the lid; a fill kernel, so that the call
// stays free of memset nodes under graph capture).
__global__ void lid_zero_kernel(double* __restrict__ a, double* __restrict__ c, int H, int W, int64_t ld) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    a[(int64_t)(H - 1) * ld + j] = 0.0;
    if (c != nullptr) c[(int64_t)(H - 1) * ld + j] = 0.0;
}

int resident_waves_of(const void* kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess)
        return 0;
    return cus * per_cu;
}

// Process-wide tuning setting, read atomically: rows per band (0: built-in).
// Any band height gives the same results.
std::atomic<int> g_pressure_band{0};

// Up to 8 levels the register-ring kernel, above that the LDS-ring one (at 8
// levels the register ring is the faster of the two).
template <int TL>
const void* pressure_kernel_of() {
    if constexpr (TL <= 8)
        return reinterpret_cast<const void*>(&pressure_stream_kernel<TL>);
    else
        return reinterpret_cast<const void*>(&pressure_stream_lds_kernel<TL>);
}

template <int TL>
void launch_pressure(const double* p, const double* b, double* out, int H, int W, int64_t ld, double cw, double cn,
                     double cb, hipStream_t s) {
    constexpr int HALO = (TL + kPV - 1) / kPV * kPV;
    constexpr int OW = 64 * kPV - 2 * HALO;
    const uint32_t strips = ceil_div(W - 64 * kPV, OW) + 1;
    int band = g_pressure_band.load(std::memory_order_relaxed);
    if (band <= 0) {
        // the tallest bands that give every resident wave slot a band (one round), at least 2*TL rows
        static const int waves = resident_waves_of(pressure_kernel_of<TL>());
        const int64_t fit = std::max<int64_t>(1, (waves > 0 ? waves : 1024) / (int64_t)strips);
        band = (int)std::max<int64_t>(2 * TL, (H - 2 + fit - 1) / fit);
    }
    const uint32_t bands = ceil_div(H - 2, band);
    if constexpr (TL <= 8)
        pressure_stream_kernel<TL><<<strips * bands, 64, 0, s>>>(p, b, out, H, W, ld, cw, cn, cb, strips, band);
    else
        pressure_stream_lds_kernel<TL><<<strips * bands, 64, 0, s>>>(p, b, out, H, W, ld, cw, cn, cb, strips, band);
}

constexpr int kMaxPressureLevels = 12;
constexpr int kDefaultPressureLevels = 12;

void launch_pressure_levels(const double* p, const double* b, double* out, int H, int W, int64_t ld, double cw,
                            double cn, double cb, int levels, hipStream_t s) {
    switch (levels) {
        case 1: launch_pressure<1>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 2: launch_pressure<2>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 3: launch_pressure<3>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 4: launch_pressure<4>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 5: launch_pressure<5>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 6: launch_pressure<6>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 7: launch_pressure<7>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 8: launch_pressure<8>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 9: launch_pressure<9>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 10: launch_pressure<10>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        case 11: launch_pressure<11>(p, b, out, H, W, ld, cw, cn, cb, s); break;
        default: launch_pressure<12>(p, b, out, H, W, ld, cw, cn, cb, s); break;
    }
}

}  // namespace
}  // namespace sten

extern "C" {

sten_status sten_cavity_pressure_f64(const double* p0, const double* b, double* out, double* work, int64_t H,
                                     int64_t W, int64_t ld, int32_t nit, double cw, double cn, double cb,
                                     int32_t levels, hipStream_t stream) {
    using namespace sten;
    if (H < 0 || W < 0 || ld < W || nit < 0 || levels < 0 || levels > kMaxPressureLevels) return STEN_ERR_ARG;
    if (H == 0 || W == 0) return STEN_OK;
    const int lev = levels == 0 ? kDefaultPressureLevels : levels;
    const int passes = nit == 0 ? 0 : (nit + lev - 1) / lev;
    const bool need_work = passes >= 2;
    const size_t span = span_bytes(H, W, ld, sizeof(double));
    if (p0 == nullptr || b == nullptr || out == nullptr || (need_work && work == nullptr)) return STEN_ERR_PTR;
    if (overlaps(p0, span, out, span) || overlaps(b, span, out, span) ||
        (need_work && (overlaps(p0, span, work, span) || overlaps(b, span, work, span) ||
                       overlaps(out, span, work, span))))
        return STEN_ERR_ALIAS;
    // the blocked kernel's layout: grid-aligned strips of 128 columns, 16-byte vectors
    if (H < 3 || W < 128 || W % 2 != 0 || ld % 2 != 0 || W * (int64_t)sizeof(double) >= ((int64_t)1 << 30) ||
        H > INT32_MAX / 2 ||
        (((uintptr_t)p0 | (uintptr_t)b | (uintptr_t)out | (need_work ? (uintptr_t)work : 0)) % 16) != 0)
        return STEN_ERR_UNSUPPORTED;
    if (!is_device_ptr(p0) || !is_device_ptr(b) || !is_device_ptr(out) || (need_work && !is_device_ptr(work)))
        return STEN_ERR_PTR;
    if (nit == 0) {
        const hipError_t e = hipMemcpy2DAsync(out, ld * sizeof(double), p0, ld * sizeof(double), W * sizeof(double),
                                              H, hipMemcpyDeviceToDevice, stream);
        return e == hipSuccess ? STEN_OK : hip_fail(e);
    }
    const int h = (int)H, w = (int)W;
    lid_zero_kernel<<<ceil_div(W, 256), 256, 0, stream>>>(out, need_work ? work : nullptr, h, w, ld);
    // pass k (1-based) applies base (+1) iterations; the last pass writes `out`
    const double* src = p0;
    const int base = nit / passes, extra = nit % passes;
    for (int k = 1; k <= passes; ++k) {
        double* dst = ((passes - k) % 2 == 0) ? out : work;
        launch_pressure_levels(src, b, dst, h, w, ld, cw, cn, cb, base + (k <= extra ? 1 : 0), stream);
        src = dst;
    }
    return check_launch();
}

sten_status sten_tune_pressure(int32_t band) {
    if (band < 0 || band > 65536) return STEN_ERR_ARG;
    sten::g_pressure_band = band;
    return STEN_OK;
}

}  // extern "C"
