// Reduced-precision form of the five-point Jacobi sweep (an extension beside
// the paper's FP64 method): grids are stored as an FP32 plane hi and an int16
// plane q with x ~ hi + q * delta(hi), delta(hi) = ulp32(hi) * 2^-16 (floored
// at 2^-149), i.e. 6 bytes per point instead of 8.
//
// One sweep per output point, all in FP32 with error-free transformations:
//   decode   each neighbour to a pair (h, l), l = q * delta(h)      (exact)
//   sum      s1,e1 = TwoSum(N.h, S.h); s2,e2 = TwoSum(s1, W.h);
//            s3,e3 = TwoSum(s2, E.h)                                (exact)
//            low = (((N.l + S.l) + W.l) + E.l) + ((e1 + e2) + e3)
//            (H, L) = TwoSum(s3, low)
//   scale    by c: exact when c is a power of two; otherwise a double-word
//            product with c = c_hi + c_lo (fmaf for the exact product error)
//   encode   q = rint(L / delta(H)); q = +32768 (not an int16) is renormalised
//            exactly: H steps to the next FP32 value up, L -= ulp(H).
// The neighbour sum keeps the listing's order N, S, W, E (Section III-A).
// Error per sweep: at most 2^-40 |H| for the re-encoding plus 17 * 2^-48 of
// the sum of neighbour magnitudes (20 * 2^-48 with a general c); FP64 is used
// only in encode and decode. The library is built with -ffp-contract=off, so
// the transformations are evaluated exactly as written.
//
// Kernel layout follows the plain sweep: a 256-lane workgroup owns ROWS output
// rows by 256*V columns, each lane streams V consecutive points (a 16-byte hi
// vector and an 8-byte q vector per row) through registers, neighbours across
// lanes come by shuffle, the wave's edge lanes load the one outside neighbour.
#include <algorithm>
#include <atomic>

#include "common.hpp"

namespace sten {
namespace {

constexpr int kBlock = 256;
constexpr size_t kPlaneAlign = 256;

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte offset of the q plane inside an encoded grid.
inline size_t q_offset(int64_t H, int64_t ld) { return align_up((size_t)(H * ld) * sizeof(float), kPlaneAlign); }

// Exponent k of delta(h) = 2^k: k = max(max(E, 1) - 127 - 23 - 16, -149), E the biased
// exponent of h; the two clamps fold into one: k = max(E, 17) - 166.
__device__ __forceinline__ int delta_exp(float h) {
    const int E = (int)((__float_as_uint(h) >> 23) & 0xFFu);
    return max(E, 17) - 166;
}

struct DW {
    float h, l;
};

__device__ __forceinline__ DW decode(float h, int16_t q) { return DW{h, ldexpf((float)q, delta_exp(h))}; }

// TwoSum (Knuth): s + e == a + b exactly, s = fl(a + b).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Re-encode a normalised pair (|L| <= half an ulp of H) as (hi, q), except
// that q may come out as +32768 (returned in qf); the caller fixes that case.
__device__ __forceinline__ float quantise(float H, float L) { return rintf(ldexpf(L, -delta_exp(H))); }

// The rare case q = +32768: move one ulp into hi (exact); the remainder
// becomes negative and fits int16.
__device__ __forceinline__ void renormalise(float& H, float L, float& qf) {
    const float ulp = ldexpf(1.0f, delta_exp(H) + 16);
    H = H + ulp;
    L = L - ulp;
    qf = quantise(H, L);
}

struct Coef {
    float hi, lo;
    int pow2;  // 1 when c is a power of two (scaling is exact)
};

// Neighbour sum and scaling of one output point; returns the normalised pair (H, L).
// POW2: c is a power of two, so scaling the pair is exact.
template <bool POW2>
__device__ __forceinline__ void stencil_point(const DW& n, const DW& s, const DW& w, const DW& e, const Coef& c,
                                              float& H, float& L) {
    float s1, e1, s2, e2, s3, e3;
    two_sum(n.h, s.h, s1, e1);
    two_sum(s1, w.h, s2, e2);
    two_sum(s2, e.h, s3, e3);
    const float lo = ((n.l + s.l) + w.l) + e.l;
    const float er = (e1 + e2) + e3;
    const float low = lo + er;
    two_sum(s3, low, H, L);
    if constexpr (POW2) {
        H = H * c.hi;
        L = L * c.hi;
    } else {
        const float p = H * c.hi;
        float ep = fmaf(H, c.hi, -p);
        ep = ep + (H * c.lo + L * c.hi);
        const float h2 = p + ep;  // Fast2Sum: |p| >= |ep|
        L = ep - (h2 - p);
        H = h2;
    }
}

template <int V>
struct HVec;
template <>
struct HVec<1> {
    typedef float hv;
    typedef int16_t qv;
};
template <>
struct HVec<4> {
    typedef float hv __attribute__((ext_vector_type(4)));
    typedef short qv __attribute__((ext_vector_type(4)));
};
template <>
struct HVec<8> {
    typedef float hv __attribute__((ext_vector_type(8)));
    typedef short qv __attribute__((ext_vector_type(8)));
};
template <>
struct HVec<16> {
    typedef float hv __attribute__((ext_vector_type(16)));
    typedef short qv __attribute__((ext_vector_type(16)));
};

template <int V, bool FULL>
__device__ __forceinline__ void load_row(const float* __restrict__ hrow, const int16_t* __restrict__ qrow, int jb,
                                         int W, DW (&d)[V]) {
    if (FULL || jb + V <= W) {
        if constexpr (V == 1) {
            d[0] = decode(hrow[jb], qrow[jb]);
        } else {
            const typename HVec<V>::hv h = *reinterpret_cast<const typename HVec<V>::hv*>(hrow + jb);
            const typename HVec<V>::qv q = *reinterpret_cast<const typename HVec<V>::qv*>(qrow + jb);
#pragma unroll
            for (int e = 0; e < V; ++e) d[e] = decode(h[e], (int16_t)q[e]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) d[e] = (jb + e < W) ? decode(hrow[jb + e], qrow[jb + e]) : DW{0.0f, 0.0f};
    }
}

template <int V>
__device__ __forceinline__ void store_row(float* __restrict__ hrow, int16_t* __restrict__ qrow, int jb, int W,
                                          const float (&h)[V], const int16_t (&q)[V]) {
    if constexpr (V > 1) {
        if (jb >= 1 && jb + V <= W - 1) {
            typename HVec<V>::hv hv;
            typename HVec<V>::qv qv;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                hv[e] = h[e];
                qv[e] = q[e];
            }
            *reinterpret_cast<typename HVec<V>::hv*>(hrow + jb) = hv;
            *reinterpret_cast<typename HVec<V>::qv*>(qrow + jb) = qv;
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const int j = jb + e;
        if (j >= 1 && j <= W - 2) {
            hrow[j] = h[e];
            qrow[j] = q[e];
        }
    }
}

__device__ __forceinline__ DW shfl_up_dw(const DW& v) { return DW{__shfl_up(v.h, 1), __shfl_up(v.l, 1)}; }
__device__ __forceinline__ DW shfl_down_dw(const DW& v) { return DW{__shfl_down(v.h, 1), __shfl_down(v.l, 1)}; }

template <int V, int ROWS, bool FULL, bool POW2>
__device__ __forceinline__ void hilo_tile(const float* __restrict__ hsrc, const int16_t* __restrict__ qsrc,
                                          float* __restrict__ hdst, int16_t* __restrict__ qdst, int n, int jb,
                                          int lane, int W, int64_t ld, const Coef& c) {
    DW r[ROWS + 2][V];
#pragma unroll
    for (int k = 0; k < ROWS + 2; ++k) {
        if (FULL || k < n + 2) {
            load_row<V, FULL>(hsrc + (int64_t)k * ld, qsrc + (int64_t)k * ld, jb, W, r[k]);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) r[k][e] = DW{0.0f, 0.0f};
        }
    }
    DW el[ROWS], er[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        el[k] = DW{0.0f, 0.0f};
        er[k] = DW{0.0f, 0.0f};
        if (FULL || k < n) {
            const int64_t off = (int64_t)(k + 1) * ld;
            if (lane == 0 && jb > 0 && jb <= W) el[k] = decode(hsrc[off + jb - 1], qsrc[off + jb - 1]);
            if (lane == kWave - 1 && jb + V < W) er[k] = decode(hsrc[off + jb + V], qsrc[off + jb + V]);
        }
    }
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        if (FULL || k < n) {  // n is uniform over the block
            DW left0 = shfl_up_dw(r[k + 1][V - 1]);
            DW rightv = shfl_down_dw(r[k + 1][0]);
            if (lane == 0) left0 = el[k];
            if (lane == kWave - 1) rightv = er[k];
            float oh[V], ol[V], qf[V];
            bool over = false;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const DW west = (e == 0) ? left0 : r[k + 1][e > 0 ? e - 1 : 0];
                const DW east = (e == V - 1) ? rightv : r[k + 1][e < V - 1 ? e + 1 : 0];
                stencil_point<POW2>(r[k][e], r[k + 2][e], west, east, c, oh[e], ol[e]);
                qf[e] = quantise(oh[e], ol[e]);
                over = over || (qf[e] > 32767.0f);
            }
            if (__any(over)) {  // rare: one branch per row for the whole wave
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if (qf[e] > 32767.0f) renormalise(oh[e], ol[e], qf[e]);
            }
            int16_t oq[V];
#pragma unroll
            for (int e = 0; e < V; ++e) oq[e] = (int16_t)qf[e];
            store_row<V>(hdst + (int64_t)k * ld, qdst + (int64_t)k * ld, jb, W, oh, oq);
        }
    }
}

// Full tile (ROWS output rows, every lane of the wave inside the grid), the
// hot path: loads address a uniform row base with 32-bit lane offsets (scalar
// base + vector offset addressing), and the two neighbours that lie in other
// waves are fetched by one load per row - lane 0 takes the left one, lane 63
// the right one - and decoded once.
template <int V, int ROWS, bool POW2>
__device__ __forceinline__ void hilo_tile_full(const float* __restrict__ hsrc, const int16_t* __restrict__ qsrc,
                                               float* __restrict__ hdst, int16_t* __restrict__ qdst, int jb,
                                               int lane, int W, int ld, const Coef& c) {
    typedef typename HVec<V>::hv HV;
    typedef typename HVec<V>::qv QV;
    HV rh[ROWS + 2];
    QV rq[ROWS + 2];
#pragma unroll
    for (int k = 0; k < ROWS + 2; ++k) {
        const int off = k * ld + jb;
        rh[k] = *reinterpret_cast<const HV*>(hsrc + off);
        rq[k] = *reinterpret_cast<const QV*>(qsrc + off);
    }
    int eidx = -1;
    if (lane == 0 && jb > 0) eidx = jb - 1;
    if (lane == kWave - 1 && jb + V < W) eidx = jb + V;
    float eh[ROWS];
    int16_t eq[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        eh[k] = 0.0f;
        eq[k] = 0;
        if (eidx >= 0) {
            const int off = (k + 1) * ld + eidx;
            eh[k] = hsrc[off];
            eq[k] = qsrc[off];
        }
    }
    DW d[ROWS + 2][V];
#pragma unroll
    for (int k = 0; k < ROWS + 2; ++k)
#pragma unroll
        for (int e = 0; e < V; ++e) d[k][e] = decode(rh[k][e], (int16_t)rq[k][e]);
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const DW edge = decode(eh[k], eq[k]);
        DW left0 = shfl_up_dw(d[k + 1][V - 1]);
        DW rightv = shfl_down_dw(d[k + 1][0]);
        if (lane == 0) left0 = edge;
        if (lane == kWave - 1) rightv = edge;
        float oh[V], ol[V], qf[V];
        bool over = false;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const DW west = (e == 0) ? left0 : d[k + 1][e > 0 ? e - 1 : 0];
            const DW east = (e == V - 1) ? rightv : d[k + 1][e < V - 1 ? e + 1 : 0];
            stencil_point<POW2>(d[k][e], d[k + 2][e], west, east, c, oh[e], ol[e]);
            qf[e] = quantise(oh[e], ol[e]);
            over = over || (qf[e] > 32767.0f);
        }
        if (__any(over)) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (qf[e] > 32767.0f) renormalise(oh[e], ol[e], qf[e]);
        }
        HV hv;
        QV qv;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            hv[e] = oh[e];
            qv[e] = (short)(int)qf[e];
        }
        const int off = k * ld + jb;
        if (jb >= 1 && jb + V <= W - 1) {
            *reinterpret_cast<HV*>(hdst + off) = hv;
            *reinterpret_cast<QV*>(qdst + off) = qv;
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int j = jb + e;
                if (j >= 1 && j <= W - 2) {
                    hdst[off + e] = oh[e];
                    qdst[off + e] = (int16_t)(int)qf[e];
                }
            }
        }
    }
}

// Streaming form of a full tile (STRIP output rows, every lane inside the
// grid, V = 4): the wave walks down its strip one row at a time and keeps the
// loads of the next D rows in flight while it computes the current row, so
// memory traffic and the (heavy) arithmetic overlap inside every wave. A
// scheduling barrier after each row keeps that order.
template <int STRIP, int D, bool POW2>
__device__ __forceinline__ void hilo_stream_full(const float* __restrict__ hsrc, const int16_t* __restrict__ qsrc,
                                                 float* __restrict__ hdst, int16_t* __restrict__ qdst, int jb,
                                                 int lane, int W, int64_t ld, const Coef& c) {
    constexpr int V = 4;
    typedef typename HVec<V>::hv HV;
    typedef typename HVec<V>::qv QV;
    constexpr int NR = STRIP + 2;  // input rows of the strip
    HV rh[NR];
    QV rq[NR];
    float elh[NR], erh[NR];
    int16_t elq[NR], erq[NR];
    const bool has_l = (lane == 0) && (jb > 0);
    const bool has_r = (lane == kWave - 1) && (jb + V < W);
    auto issue = [&](int k) {
        const int64_t off = (int64_t)k * ld;
        rh[k] = *reinterpret_cast<const HV*>(hsrc + off + jb);
        rq[k] = *reinterpret_cast<const QV*>(qsrc + off + jb);
        elh[k] = 0.0f;
        elq[k] = 0;
        erh[k] = 0.0f;
        erq[k] = 0;
        if (k >= 1 && k <= STRIP) {  // only rows that serve as the middle row need side neighbours
            if (has_l) {
                elh[k] = hsrc[off + jb - 1];
                elq[k] = qsrc[off + jb - 1];
            }
            if (has_r) {
                erh[k] = hsrc[off + jb + V];
                erq[k] = qsrc[off + jb + V];
            }
        }
    };
#pragma unroll
    for (int k = 0; k < (D + 2 < NR ? D + 2 : NR); ++k) issue(k);
    DW up[V], mid[V], dn[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        up[e] = decode(rh[0][e], (int16_t)rq[0][e]);
        mid[e] = decode(rh[1][e], (int16_t)rq[1][e]);
    }
    DW midl = decode(elh[1], elq[1]);
    DW midr = decode(erh[1], erq[1]);
#pragma unroll
    for (int k = 0; k < STRIP; ++k) {
        if (k + D + 2 < NR) issue(k + D + 2);
#pragma unroll
        for (int e = 0; e < V; ++e) dn[e] = decode(rh[k + 2][e], (int16_t)rq[k + 2][e]);
        DW left0 = shfl_up_dw(mid[V - 1]);
        DW rightv = shfl_down_dw(mid[0]);
        if (lane == 0) left0 = midl;
        if (lane == kWave - 1) rightv = midr;
        float oh[V], ol[V], qf[V];
        bool over = false;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const DW west = (e == 0) ? left0 : mid[e > 0 ? e - 1 : 0];
            const DW east = (e == V - 1) ? rightv : mid[e < V - 1 ? e + 1 : 0];
            stencil_point<POW2>(up[e], dn[e], west, east, c, oh[e], ol[e]);
            qf[e] = quantise(oh[e], ol[e]);
            over = over || (qf[e] > 32767.0f);
        }
        if (__any(over)) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (qf[e] > 32767.0f) renormalise(oh[e], ol[e], qf[e]);
        }
        int16_t oq[V];
#pragma unroll
        for (int e = 0; e < V; ++e) oq[e] = (int16_t)qf[e];
        store_row<V>(hdst + (int64_t)k * ld, qdst + (int64_t)k * ld, jb, W, oh, oq);
        if (k + 2 < NR) {
            midl = decode(elh[k + 2 < NR ? k + 2 : 0], elq[k + 2 < NR ? k + 2 : 0]);
            midr = decode(erh[k + 2 < NR ? k + 2 : 0], erq[k + 2 < NR ? k + 2 : 0]);
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            up[e] = mid[e];
            mid[e] = dn[e];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int STRIP, int D, bool POW2>
__global__ __launch_bounds__(kBlock) void hilo_stream_kernel(const float* __restrict__ hin,
                                                             const int16_t* __restrict__ qin,
                                                             float* __restrict__ hout, int16_t* __restrict__ qout,
                                                             int H, int W, int64_t ld, Coef c, uint32_t tiles_x) {
    constexpr int V = 4;
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t ty = tile / tiles_x;
    const uint32_t tx = tile - ty * tiles_x;
    const int lane = threadIdx.x & (kWave - 1);
    const int jb = ((int)tx * kBlock + (int)threadIdx.x) * V;
    const int i0 = 1 + (int)ty * STRIP;
    const int n = min(STRIP, H - 1 - i0);
    const int wave_end = (jb - lane * V) + kWave * V;
    if (n == STRIP && wave_end <= W) {
        const int64_t in_off = (int64_t)(i0 - 1) * ld;
        const int64_t out_off = (int64_t)i0 * ld;
        hilo_stream_full<STRIP, D, POW2>(hin + in_off, qin + in_off, hout + out_off, qout + out_off, jb, lane, W,
                                         ld, c);
    } else {
        // ragged strip: 4-row guarded tiles
        for (int s0 = 0; s0 < n; s0 += 4) {
            const int m = min(4, n - s0);
            const int64_t in_off = (int64_t)(i0 + s0 - 1) * ld;
            const int64_t out_off = (int64_t)(i0 + s0) * ld;
            hilo_tile<V, 4, false, POW2>(hin + in_off, qin + in_off, hout + out_off, qout + out_off, m, jb, lane, W,
                                         ld, c);
        }
    }
}

template <int V, int ROWS, bool POW2>
__global__ __launch_bounds__(kBlock) void hilo_sweep_kernel(const float* __restrict__ hin,
                                                            const int16_t* __restrict__ qin,
                                                            float* __restrict__ hout, int16_t* __restrict__ qout,
                                                            int H, int W, int64_t ld, Coef c, uint32_t tiles_x) {
    const uint32_t tile = xcd_tile_of_block(blockIdx.x, gridDim.x);
    const uint32_t ty = tile / tiles_x;
    const uint32_t tx = tile - ty * tiles_x;
    const int lane = threadIdx.x & (kWave - 1);
    const int jb = ((int)tx * kBlock + (int)threadIdx.x) * V;
    const int i0 = 1 + (int)ty * ROWS;
    const int n = min(ROWS, H - 1 - i0);
    const int wave_end = (jb - lane * V) + kWave * V;
    const int64_t in_off = (int64_t)(i0 - 1) * ld;
    const int64_t out_off = (int64_t)i0 * ld;
    if (n == ROWS && wave_end <= W) {
        if constexpr (V >= 4)
            hilo_tile_full<V, ROWS, POW2>(hin + in_off, qin + in_off, hout + out_off, qout + out_off, jb, lane, W,
                                          (int)ld, c);
        else
            hilo_tile<V, ROWS, true, POW2>(hin + in_off, qin + in_off, hout + out_off, qout + out_off, n, jb, lane,
                                           W, ld, c);
    } else
        hilo_tile<V, ROWS, false, POW2>(hin + in_off, qin + in_off, hout + out_off, qout + out_off, n, jb, lane, W, ld, c);
}

// FP64 -> (hi, q) for every point; when h2/q2 are given, the ring also goes there.
// Encode one value: h = RN32(v), q = rint((v - h) / delta(h)); the one q that
// int16 cannot hold (+32768) moves h up one ulp and q to the remainder.
__device__ __forceinline__ void encode_one(double v, float& h, int16_t& qq) {
    h = (float)v;
    int k = delta_exp(h);
    double qd = rint(ldexp(v - (double)h, -k));
    if (qd > 32767.0) {
        h = nextafterf(h, INFINITY);
        k = delta_exp(h);
        qd = rint(ldexp(v - (double)h, -k));
    }
    qq = (int16_t)qd;
}

__device__ __forceinline__ double decode_one(float h, int16_t q) { return (double)h + ldexp((double)q, delta_exp(h)); }

// Element-wise encode for any layout. When h2 is given the ring also goes
// there (the second ping-pong grid of the FP64-in, FP64-out call).
__global__ void hilo_encode_kernel(const double* __restrict__ x, float* __restrict__ hi, int16_t* __restrict__ q,
                                   float* __restrict__ h2, int16_t* __restrict__ q2, int H, int W, int64_t ld) {
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / W;
        const int64_t j = idx - i * W;
        const int64_t off = i * ld + j;
        float h;
        int16_t qq;
        encode_one(x[off], h, qq);
        hi[off] = h;
        q[off] = qq;
        if (h2 != nullptr && (i == 0 || i == H - 1 || j == 0 || j == W - 1)) {
            h2[off] = h;
            q2[off] = qq;
        }
    }
}

// (hi, q) -> FP64; ring points come from ring_src when it is given.
__global__ void hilo_decode_kernel(const float* __restrict__ hi, const int16_t* __restrict__ q,
                                   double* __restrict__ x, const double* __restrict__ ring_src, int H, int W,
                                   int64_t ld) {
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / W;
        const int64_t j = idx - i * W;
        const int64_t off = i * ld + j;
        if (ring_src != nullptr && (i == 0 || i == H - 1 || j == 0 || j == W - 1)) {
            x[off] = ring_src[off];
        } else {
            x[off] = decode_one(hi[off], q[off]);
        }
    }
}

// Vector forms of encode and decode (ld a multiple of 4, x 16-byte aligned;
// the planes are 256-byte aligned): a lane takes 4 consecutive elements of a
// row, as two 16-byte loads or stores of x, one 16-byte of hi and 8 bytes of
// q; workgroups along blockIdx.x cover a row, blockIdx.y walks the rows. No
// division per element. Same per-element steps as the element-wise kernels.
constexpr int kCodeBlock = 256;
typedef double D2 __attribute__((ext_vector_type(2)));
typedef float F4 __attribute__((ext_vector_type(4)));
typedef short S4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kCodeBlock) void hilo_encode_vec_kernel(const double* __restrict__ x,
                                                                     float* __restrict__ hi, int16_t* __restrict__ q,
                                                                     float* __restrict__ h2, int16_t* __restrict__ q2,
                                                                     int H, int W, int64_t ld) {
    const int j = ((int)blockIdx.x * kCodeBlock + (int)threadIdx.x) * 4;
    if (j >= W) return;
    for (int64_t i = blockIdx.y; i < H; i += gridDim.y) {
        const int64_t off = i * ld + j;
        const bool ring_row = i == 0 || i == H - 1;
        if (j + 4 <= W) {
            const D2 a = *reinterpret_cast<const D2*>(x + off);
            const D2 b = *reinterpret_cast<const D2*>(x + off + 2);
            const double v[4] = {a[0], a[1], b[0], b[1]};
            F4 hv;
            S4 qv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float h;
                int16_t qq;
                encode_one(v[e], h, qq);
                hv[e] = h;
                qv[e] = qq;
            }
            *reinterpret_cast<F4*>(hi + off) = hv;
            *reinterpret_cast<S4*>(q + off) = qv;
            if (h2 != nullptr) {
                if (ring_row) {
                    *reinterpret_cast<F4*>(h2 + off) = hv;
                    *reinterpret_cast<S4*>(q2 + off) = qv;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (j + e == 0 || j + e == W - 1) {
                            h2[off + e] = hv[e];
                            q2[off + e] = qv[e];
                        }
                    }
                }
            }
        } else {
            for (int e = 0; e < W - j; ++e) {
                float h;
                int16_t qq;
                encode_one(x[off + e], h, qq);
                hi[off + e] = h;
                q[off + e] = qq;
                if (h2 != nullptr && (ring_row || j + e == 0 || j + e == W - 1)) {
                    h2[off + e] = h;
                    q2[off + e] = qq;
                }
            }
        }
    }
}

__global__ __launch_bounds__(kCodeBlock) void hilo_decode_vec_kernel(const float* __restrict__ hi,
                                                                     const int16_t* __restrict__ q,
                                                                     double* __restrict__ x,
                                                                     const double* __restrict__ ring_src, int H,
                                                                     int W, int64_t ld) {
    const int j = ((int)blockIdx.x * kCodeBlock + (int)threadIdx.x) * 4;
    if (j >= W) return;
    for (int64_t i = blockIdx.y; i < H; i += gridDim.y) {
        const int64_t off = i * ld + j;
        const bool ring_row = ring_src != nullptr && (i == 0 || i == H - 1);
        if (j + 4 <= W) {
            D2 a, b;
            if (ring_row) {
                a = *reinterpret_cast<const D2*>(ring_src + off);
                b = *reinterpret_cast<const D2*>(ring_src + off + 2);
            } else {
                const F4 hv = *reinterpret_cast<const F4*>(hi + off);
                const S4 qv = *reinterpret_cast<const S4*>(q + off);
                double v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    v[e] = (ring_src != nullptr && (j + e == 0 || j + e == W - 1)) ? ring_src[off + e]
                                                                                     : decode_one(hv[e], qv[e]);
                a = D2{v[0], v[1]};
                b = D2{v[2], v[3]};
            }
            *reinterpret_cast<D2*>(x + off) = a;
            *reinterpret_cast<D2*>(x + off + 2) = b;
        } else {
            for (int e = 0; e < W - j; ++e)
                x[off + e] = (ring_src != nullptr && (ring_row || j + e == 0 || j + e == W - 1))
                                 ? ring_src[off + e]
                                 : decode_one(hi[off + e], q[off + e]);
        }
    }
}

inline uint32_t code_blocks(int64_t total) {
    return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
}

inline bool code_vec_ok(const void* x, int64_t ld) { return ((uintptr_t)x % 16) == 0 && ld % 4 == 0; }

inline dim3 code_grid(int64_t H, int64_t W) {
    return dim3(ceil_div(W, (int64_t)kCodeBlock * 4), (uint32_t)std::min<int64_t>(H, 65535));
}

void launch_encode(const double* x, float* hi, int16_t* q, float* h2, int16_t* q2, int H, int W, int64_t ld,
                   hipStream_t s) {
    if (code_vec_ok(x, ld))
        hilo_encode_vec_kernel<<<code_grid(H, W), kCodeBlock, 0, s>>>(x, hi, q, h2, q2, H, W, ld);
    else
        hilo_encode_kernel<<<code_blocks((int64_t)H * W), 256, 0, s>>>(x, hi, q, h2, q2, H, W, ld);
}

void launch_decode(const float* hi, const int16_t* q, double* x, const double* ring_src, int H, int W, int64_t ld,
                   hipStream_t s) {
    if (code_vec_ok(x, ld) && (ring_src == nullptr || ((uintptr_t)ring_src % 16) == 0))
        hilo_decode_vec_kernel<<<code_grid(H, W), kCodeBlock, 0, s>>>(hi, q, x, ring_src, H, W, ld);
    else
        hilo_decode_kernel<<<code_blocks((int64_t)H * W), 256, 0, s>>>(hi, q, x, ring_src, H, W, ld);
}

// Copy the encoded ring (or the whole grid when `full`) from (hs, qs) to (hd, qd) and (hd2, qd2).
__global__ void hilo_copy_kernel(const float* __restrict__ hs, const int16_t* __restrict__ qs,
                                 float* __restrict__ hd, int16_t* __restrict__ qd, float* __restrict__ hd2,
                                 int16_t* __restrict__ qd2, int H, int W, int64_t ld, int full) {
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / W;
        const int64_t j = idx - i * W;
        if (!full && !(i == 0 || i == H - 1 || j == 0 || j == W - 1)) continue;
        const int64_t off = i * ld + j;
        const float h = hs[off];
        const int16_t qq = qs[off];
        hd[off] = h;
        qd[off] = qq;
        if (hd2 != nullptr) {
            hd2[off] = h;
            qd2[off] = qq;
        }
    }
}

struct Planes {
    float* h;
    int16_t* q;
};

inline Planes planes(void* base, int64_t H, int64_t ld) {
    char* b = (char*)base;
    return Planes{(float*)b, (int16_t*)(b + q_offset(H, ld))};
}

inline uint32_t grid_blocks(int64_t total) { return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536)); }

Coef make_coef(double c) {
    Coef k;
    k.hi = (float)c;
    k.lo = (float)(c - (double)k.hi);
    int e = 0;
    const double m = frexp(c, &e);
    k.pow2 = (c != 0.0 && (m == 0.5 || m == -0.5) && k.lo == 0.0f) ? 1 : 0;
    return k;
}

// Process-wide variant setting, read atomically once per call; both variants
// compute the same bits.
std::atomic<int> g_hilo_variant{0};

template <int V, int ROWS>
void launch_hilo_rows(const Planes& in, const Planes& out, int H, int W, int64_t ld, const Coef& c, hipStream_t s) {
    const uint32_t tiles_x = ceil_div(W, (int64_t)kBlock * V);
    const uint32_t tiles_y = ceil_div(H - 2, ROWS);
    if (c.pow2)
        hilo_sweep_kernel<V, ROWS, true><<<tiles_x * tiles_y, kBlock, 0, s>>>(in.h, in.q, out.h, out.q, H, W, ld, c,
                                                                              tiles_x);
    else
        hilo_sweep_kernel<V, ROWS, false><<<tiles_x * tiles_y, kBlock, 0, s>>>(in.h, in.q, out.h, out.q, H, W, ld, c,
                                                                               tiles_x);
}

template <int STRIP, int D>
void launch_hilo_stream(const Planes& in, const Planes& out, int H, int W, int64_t ld, const Coef& c, hipStream_t s) {
    const uint32_t tiles_x = ceil_div(W, (int64_t)kBlock * 4);
    const uint32_t tiles_y = ceil_div(H - 2, STRIP);
    if (c.pow2)
        hilo_stream_kernel<STRIP, D, true><<<tiles_x * tiles_y, kBlock, 0, s>>>(in.h, in.q, out.h, out.q, H, W, ld,
                                                                                c, tiles_x);
    else
        hilo_stream_kernel<STRIP, D, false><<<tiles_x * tiles_y, kBlock, 0, s>>>(in.h, in.q, out.h, out.q, H, W, ld,
                                                                                 c, tiles_x);
}

// Kernel variants (tuning hook): 1: tiles of 4 rows x 4 points per lane;
// 2: 8 rows x 4 points; 3: 4 rows x 8 points; 4: 2 rows x 8 points;
// 5: row streaming over 16-row strips (loads 4 rows ahead); 6: 32-row strips;
// 7: 2 rows x 4 points; 8: 1 row x 8 points; 9: 1 row x 16 points; 10: 3 rows x 8 points.
constexpr int kHiloDefaultVariant = 4;

template <int V, int ROWS>
bool launch_tile_if_aligned(const Planes& in, const Planes& out, int H, int W, int64_t ld, const Coef& c,
                            hipStream_t s) {
    if (ld % V != 0) return false;
    launch_hilo_rows<V, ROWS>(in, out, H, W, ld, c, s);
    return true;
}

void launch_hilo(const Planes& in, const Planes& out, int H, int W, int64_t ld, const Coef& c, int variant,
                 hipStream_t s) {
    // 32-bit lane offsets inside a tile need (rows + 2) * ld well below 2^31
    if (ld <= (int64_t(1) << 26)) {
        switch (variant) {
            case 2: if (launch_tile_if_aligned<4, 8>(in, out, H, W, ld, c, s)) return; break;
            case 3: if (launch_tile_if_aligned<8, 4>(in, out, H, W, ld, c, s)) return; break;
            case 4: if (launch_tile_if_aligned<8, 2>(in, out, H, W, ld, c, s)) return; break;
            case 5: if (ld % 4 == 0) { launch_hilo_stream<16, 4>(in, out, H, W, ld, c, s); return; } break;
            case 6: if (ld % 4 == 0) { launch_hilo_stream<32, 4>(in, out, H, W, ld, c, s); return; } break;
            case 7: if (launch_tile_if_aligned<4, 2>(in, out, H, W, ld, c, s)) return; break;
            case 8: if (launch_tile_if_aligned<8, 1>(in, out, H, W, ld, c, s)) return; break;
            case 9: if (launch_tile_if_aligned<16, 1>(in, out, H, W, ld, c, s)) return; break;
            case 10: if (launch_tile_if_aligned<8, 3>(in, out, H, W, ld, c, s)) return; break;
            default: break;
        }
        if (launch_tile_if_aligned<4, 4>(in, out, H, W, ld, c, s)) return;
    }
    launch_hilo_rows<1, 4>(in, out, H, W, ld, c, s);
}

size_t hilo_bytes(int64_t H, int64_t ld) {
    if (H <= 0 || ld <= 0) return 0;
    return q_offset(H, ld) + align_up((size_t)(H * ld) * sizeof(int16_t), kPlaneAlign);
}

sten_status check_hilo_ptr(const void* p) {
    if (p == nullptr) return STEN_ERR_PTR;
    if ((uintptr_t)p % kPlaneAlign != 0) return STEN_ERR_ARG;
    return STEN_OK;
}

sten_status check_sizes(int64_t H, int64_t W, int64_t ld, int32_t T) {
    if (H < 0 || W < 0 || T < 0) return STEN_ERR_ARG;
    if (H > 0 && ld < W) return STEN_ERR_ARG;
    if (H > INT32_MAX - 2 || W > INT32_MAX - 2) return STEN_ERR_ARG;
    return STEN_OK;
}

// T encoded sweeps from `src` (read only) into `dst`, `work` second buffer.
sten_status run_hilo_sweeps(const Planes& src, const Planes& dst, const Planes& work, int H, int W, int64_t ld,
                            int32_t T, const Coef& c, hipStream_t stream) {
    const int64_t total = (int64_t)H * W;
    if (T == 0 || H < 3 || W < 3) {
        hilo_copy_kernel<<<grid_blocks(total), 256, 0, stream>>>(src.h, src.q, dst.h, dst.q, nullptr, nullptr, H, W,
                                                                 ld, 1);
        return check_launch();
    }
    const bool need_work = T >= 2;
    hilo_copy_kernel<<<grid_blocks(total), 256, 0, stream>>>(src.h, src.q, dst.h, dst.q,
                                                             need_work ? work.h : nullptr,
                                                             need_work ? work.q : nullptr, H, W, ld, 0);
    const int variant_set = g_hilo_variant.load(std::memory_order_relaxed);
    const int variant = variant_set > 0 ? variant_set : kHiloDefaultVariant;
    Planes cur = src;
    for (int32_t k = 1; k <= T; ++k) {
        const Planes& d = ((T - k) % 2 == 0) ? dst : work;
        launch_hilo(cur, d, H, W, ld, c, variant, stream);
        cur = d;
    }
    return check_launch();
}

}  // namespace
}  // namespace sten

extern "C" {

size_t sten_hilo_bytes(int64_t H, int64_t ld) { return sten::hilo_bytes(H, ld); }

size_t sten_jacobi5_f64_hilo_work_bytes(int64_t H, int64_t ld) { return 2 * sten::hilo_bytes(H, ld); }

sten_status sten_hilo_encode(const double* x, void* hilo, int64_t H, int64_t W, int64_t ld, hipStream_t stream) {
    using namespace sten;
    sten_status st = check_sizes(H, W, ld, 0);
    if (st != STEN_OK || H == 0 || W == 0) return st;
    if (x == nullptr) return STEN_ERR_PTR;
    if ((st = check_hilo_ptr(hilo)) != STEN_OK) return st;
    if (overlaps(x, span_bytes(H, W, ld, 8), hilo, hilo_bytes(H, ld))) return STEN_ERR_ALIAS;
    if (!is_device_ptr(x) || !is_device_ptr(hilo)) return STEN_ERR_PTR;
    const Planes p = planes(hilo, H, ld);
    launch_encode(x, p.h, p.q, nullptr, nullptr, (int)H, (int)W, ld, stream);
    return check_launch();
}

sten_status sten_hilo_decode(const void* hilo, double* x, int64_t H, int64_t W, int64_t ld, hipStream_t stream) {
    using namespace sten;
    sten_status st = check_sizes(H, W, ld, 0);
    if (st != STEN_OK || H == 0 || W == 0) return st;
    if (x == nullptr) return STEN_ERR_PTR;
    if ((st = check_hilo_ptr(hilo)) != STEN_OK) return st;
    if (overlaps(x, span_bytes(H, W, ld, 8), hilo, hilo_bytes(H, ld))) return STEN_ERR_ALIAS;
    if (!is_device_ptr(x) || !is_device_ptr(hilo)) return STEN_ERR_PTR;
    const Planes p = planes((void*)hilo, H, ld);
    launch_decode(p.h, p.q, x, nullptr, (int)H, (int)W, ld, stream);
    return check_launch();
}

sten_status sten_jacobi5_hilo(const void* src, void* dst, void* work, int64_t H, int64_t W, int64_t ld, int32_t T,
                              double c, hipStream_t stream) {
    using namespace sten;
    sten_status st = check_sizes(H, W, ld, T);
    if (st != STEN_OK || H == 0 || W == 0) return st;
    const bool need_work = T >= 2 && H >= 3 && W >= 3;
    if ((st = check_hilo_ptr(src)) != STEN_OK || (st = check_hilo_ptr(dst)) != STEN_OK) return st;
    if (need_work && (st = check_hilo_ptr(work)) != STEN_OK) return st;
    const size_t nb = hilo_bytes(H, ld);
    if (overlaps(src, nb, dst, nb)) return STEN_ERR_ALIAS;
    if (need_work && (overlaps(src, nb, work, nb) || overlaps(dst, nb, work, nb))) return STEN_ERR_ALIAS;
    if (!is_device_ptr(src) || !is_device_ptr(dst) || (need_work && !is_device_ptr(work))) return STEN_ERR_PTR;
    const Planes w = need_work ? planes(work, H, ld) : Planes{nullptr, nullptr};
    return run_hilo_sweeps(planes((void*)src, H, ld), planes(dst, H, ld), w, (int)H, (int)W, ld, T, make_coef(c),
                           stream);
}

sten_status sten_jacobi5_f64_hilo(const double* u0, double* out, void* work, size_t work_bytes, int64_t H, int64_t W,
                                  int64_t ld, int32_t T, double c, hipStream_t stream) {
    using namespace sten;
    sten_status st = check_sizes(H, W, ld, T);
    if (st != STEN_OK || H == 0 || W == 0) return st;
    if (u0 == nullptr || out == nullptr) return STEN_ERR_PTR;
    if ((st = check_hilo_ptr(work)) != STEN_OK) return st;
    const size_t nb = hilo_bytes(H, ld);
    if (work_bytes < 2 * nb) return STEN_ERR_WORKSPACE;
    const size_t ng = span_bytes(H, W, ld, 8);
    if (overlaps(u0, ng, out, ng) || overlaps(u0, ng, work, 2 * nb) || overlaps(out, ng, work, 2 * nb))
        return STEN_ERR_ALIAS;
    if (!is_device_ptr(u0) || !is_device_ptr(out) || !is_device_ptr(work)) return STEN_ERR_PTR;
    const Planes a = planes(work, H, ld);
    const Planes b = planes((char*)work + nb, H, ld);
    const int h = (int)H, w = (int)W;
    // encode u0 into a (whole grid) and its ring into b
    launch_encode(u0, a.h, a.q, b.h, b.q, h, w, ld, stream);
    Planes cur = a;
    if (T > 0 && H >= 3 && W >= 3) {
        const Coef k = make_coef(c);
        const int variant_set = g_hilo_variant.load(std::memory_order_relaxed);
        const int variant = variant_set > 0 ? variant_set : kHiloDefaultVariant;
        for (int32_t s = 0; s < T; ++s) {
            const Planes& d = (s % 2 == 0) ? b : a;
            launch_hilo(cur, d, h, w, ld, k, variant, stream);
            cur = d;
        }
    }
    launch_decode(cur.h, cur.q, out, u0, h, w, ld, stream);
    return check_launch();
}

// Tuning hook: kernel variant of the hi/lo sweep (1..10; 0 = built-in).
sten_status sten_tune_hilo_variant(int32_t variant) {
    if (variant < 0 || variant > 10) return STEN_ERR_ARG;
    sten::g_hilo_variant = variant;
    return STEN_OK;
}

}  // extern "C"
