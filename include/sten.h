/*
 * sten.h - C ABI of libsten, the MI355X (gfx950) library for the 2-D
 * five-point Jacobi (Laplace) sweep.
 *
 * The method (listing of the 2-D Laplace solver, Section III-A of "An
 * Adaptive Distributed Stencil Abstraction for GPUs"): two same-shape grids
 * carry the same boundary ring; each iteration writes every interior point of
 * one grid from the other as
 *     c * (((N + S) + W) + E)
 * (N = row above, S = row below, W = left column, E = right column; the sum is
 * evaluated left to right and multiplied once by c, 0.25 in the paper), then
 * the two grids swap roles. The ring is never written. An assignment whose
 * right side reads its own output is rejected (Section III-A), which here is
 * the rule that no two buffers of a call may overlap.
 *
 * Conventions shared by every call:
 *   - Grids are row-major: element (i, j) sits at p[i * ld + j], i in [0, H)
 *     rows, j in [0, W) columns, row stride ld >= W elements. All grids of one
 *     call share H, W and ld.
 *   - All grid pointers are DEVICE memory on the current HIP device, owned by
 *     the caller. The library never allocates or frees device memory; scratch
 *     space ("work") is passed in.
 *   - Every call only enqueues work on `stream` and returns without
 *     synchronising. A kernel fault surfaces at the caller's next
 *     synchronisation, not in the returned status.
 *   - Arguments are checked before anything is enqueued. On any error nothing
 *     is enqueued and no output is touched.
 *   - Degenerate grids: H < 3 or W < 3 (empty interior) or T == 0 copy the
 *     input to the output (NumPy's empty-slice semantics). H == 0 or W == 0
 *     is a valid no-op.
 *   - Results are deterministic: the same inputs give the same bits.
 */
#ifndef STEN_H
#define STEN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STEN_OK = 0,
    STEN_ERR_ARG = -1,         /* H, W, T < 0; ld < W; count/size out of range */
    STEN_ERR_ALIAS = -2,       /* two buffers of the call overlap (Section III-A rule) */
    STEN_ERR_PTR = -3,         /* a required pointer is NULL or not device memory of the current device */
    STEN_ERR_WORKSPACE = -4,   /* workspace smaller than the matching *_bytes() query */
    STEN_ERR_HIP = -5,         /* a HIP call failed; see sten_last_hip_error() */
    STEN_ERR_UNSUPPORTED = -6  /* valid request this build does not handle (stated per call) */
} sten_status;

/* Human-readable name of a status code (static string, never NULL). */
const char* sten_status_string(sten_status s);

/* hipError_t of the most recent STEN_ERR_HIP returned on the calling thread. */
int sten_last_hip_error(void);

/* ------------------------------------------------------------------------ */
/* Plain method (Section III-A listing; iteration counts of Section V)       */
/* ------------------------------------------------------------------------ */

/*
 * T sweeps of the method in FP64, starting from u0; the result lands in out.
 *   u0   [in]  H x W grid (stride ld); never written.
 *   out  [out] H x W grid: the grid after T sweeps, ring equal to u0's ring.
 *   work [tmp] H x W grid used as the second buffer of the ping-pong; its
 *              contents on return are unspecified. Needed when T >= 2 and the
 *              interior is non-empty; may be NULL otherwise.
 *   c          coefficient of the sweep (0.25 in the paper).
 * Bit-exact with the sweep evaluated in FP64 in the listing's order (no fused
 * multiply-add, no reassociation). Errors: STEN_ERR_ARG, STEN_ERR_PTR,
 * STEN_ERR_ALIAS (any two of u0, out, work overlap), STEN_ERR_HIP.
 */
sten_status sten_jacobi5_f64(const double* u0, double* out, double* work,
                             int64_t H, int64_t W, int64_t ld, int32_t T, double c,
                             hipStream_t stream);

/* The same method in FP32 (c is used as given, in FP32). Bit-exact with the
 * listing's expression evaluated in FP32 round-to-nearest. Same errors. */
sten_status sten_jacobi5_f32(const float* u0, float* out, float* work,
                             int64_t H, int64_t W, int64_t ld, int32_t T, float c,
                             hipStream_t stream);

/*
 * One sweep (the kernel of one iteration node; Section III-C executes one
 * such kernel per node): the interior of dst from src. dst's ring is not
 * touched. src and dst must not overlap (STEN_ERR_ALIAS). Grids with an
 * empty interior are a no-op. Same bit-exactness as sten_jacobi5_f64.
 */
sten_status sten_sweep_f64(const double* src, double* dst, int64_t H, int64_t W, int64_t ld, double c,
                           hipStream_t stream);
sten_status sten_sweep_f32(const float* src, float* dst, int64_t H, int64_t W, int64_t ld, float c,
                           hipStream_t stream);

/* Tuning hook: output rows per workgroup tile of the sweep kernels (4, 8 or
 * 16; 0 restores the built-in choice). Process-wide; not thread-safe against
 * concurrent launches. STEN_ERR_ARG for other values. */
sten_status sten_tune_sweep_rows(int32_t rows);

/* ------------------------------------------------------------------------ */
/* Library introspection (host only; no GPU needed)                          */
/* ------------------------------------------------------------------------ */

/* Workgroup index -> tile index map used by the sweep launches: hardware
 * hands workgroup b to XCD (b mod 8); this map gives each XCD a contiguous
 * band of tiles so vertical neighbours share that XCD's L2. Bijective on
 * [0, nb). Exposed so that host tests can check it. */
uint32_t sten_xcd_tile_of_block(uint32_t b, uint32_t nb);

/* Library version string. */
const char* sten_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STEN_H */
