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
 *   - Tuning settings (sten_tune_*) are process-wide. Each is stored and read
 *     atomically, and every value a setter accepts gives the same results
 *     (they change speed only), so calls may run in several threads while a
 *     setter runs: a call then uses some mix of the old and new settings and
 *     still computes the method.
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

/*
 * Operations whose caller-provided device workspace sten_workspace_bytes
 * sizes. The backend works only on buffers its caller owns (the paper's data
 * layout gives each chare its own arrays, Section III-C), so every call that
 * needs scratch space takes it as an argument; this is the one query for how
 * much.
 */
typedef enum {
    STEN_OP_F64 = 0,    /* sten_jacobi5_f64: the `work` grid (FP64) */
    STEN_OP_F32 = 1,    /* sten_jacobi5_f32: the `work` grid (FP32) */
    STEN_OP_HILO = 2,   /* sten_jacobi5_f64_hilo: `work` (two encoded grids) */
    STEN_OP_BATCH = 3,  /* sten_batch_plan: `dev_ws`, with H = number of grids (W, T ignored) */
    STEN_OP_ADJ = 4,    /* sten_jacobi5_adjoint_f32: the `work` grid (FP32) */
    STEN_OP_STATES = 5  /* sten_jacobi5_f32_states: the T + 1 recorded FP32 grids */
} sten_op;

/* Value sten_workspace_bytes returns for an unknown op or invalid sizes. */
#define STEN_WORKSPACE_INVALID ((size_t)-1)

/*
 * Bytes of device workspace `op` needs on an H x W grid with row stride
 * ld = W (a wider stride needs H * ld elements per grid instead) and T
 * sweeps. 0 when the call needs none: T < 2 or an empty interior for the
 * plain and adjoint grids, H == 0 or W == 0 otherwise. STEN_WORKSPACE_INVALID
 * for an unknown op, H, W or T negative, H or W above 2^30, or a size past
 * SIZE_MAX. Pure host function; no HIP call.
 */
size_t sten_workspace_bytes(int op, int64_t H, int64_t W, int32_t T);

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
 * multiply-add, no reassociation). Schedule: when the three grids are 16-byte
 * aligned with an even ld and T >= 2, several sweeps run per launch
 * (temporal blocking, at most 12-14 (FP64) or 8-12 (FP32) by grid size by
 * default, T split evenly over the launches; see sten_tune_schedule), else one sweep
 * per launch; both give the same bits. Errors: STEN_ERR_ARG, STEN_ERR_PTR,
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

/* The listing's loop on two arrays (Section III-A): m sweeps with coefficient c
 * ping-ponging between a and b, starting from a (sweep 1 reads a and writes
 * b's interior, sweep k reads the array sweep k-1 wrote). Afterwards the array
 * sweep m wrote holds iterate m and the other holds iterate m-1, exactly as
 * after m single sweeps, PROVIDED the rings of a and b hold the same values (a
 * sweep never writes a ring, so with equal rings every level of a blocked
 * launch sees the ring the single sweep would). The first m-1 sweeps run as
 * blocked launches of up to the plain schedule's levels (sten_tune_schedule),
 * the last as one sweep. a, b: H x W FP64, row stride ld, device memory, not
 * overlapping (STEN_ERR_ALIAS). m = 0 or an empty interior: no-op. Rows of
 * 2^27 elements or more, odd ld or unaligned data run as single sweeps. */
sten_status sten_sweep_chain_f64(double* a, double* b, int64_t H, int64_t W, int64_t ld, int32_t m, double c,
                                 hipStream_t stream);

/* The same m sweeps when iterate m-1 is not needed afterwards (the lazy
 * frontend uses it when the next recorded node overwrites the other array's
 * whole interior, Section III-B). All m sweeps run as the fewest blocked
 * launches the plain schedule allows (sten_tune_schedule); iterate m lands in
 * the array the last of them writes, with the same bits as
 * sten_sweep_chain_f64, and *lands_in_b (host memory, written before the call
 * returns) says which: 1 for b, 0 for a. The other array's interior is left
 * unspecified; both rings are untouched. Without blocked launches (see
 * sten_sweep_chain_f64) iterate m lands as after m single sweeps (b for odd
 * m). lands_in_b NULL: STEN_ERR_PTR; other arguments, checks and status codes
 * as sten_sweep_chain_f64. */
sten_status sten_sweep_chain_last_f64(double* a, double* b, int64_t H, int64_t W, int64_t ld, int32_t m, double c,
                                      int32_t* lands_in_b, hipStream_t stream);

/*
 * Temporal blocking (the same method, a different schedule): each launch
 * applies up to `levels` sweeps while reading and writing the grid once, so one
 * pass over HBM serves several sweeps (the T sweeps are split as evenly as
 * ceil(T / levels) launches allow). Two kernels (sten_tune_tb picks one):
 *  - streaming (built-in, levels 1..12; FP64 also 13 and 14, at 2 waves per
 *    SIMD instead of 3): one wave walks down a band of rows
 *    and keeps, for every level, the last two rows it produced; each row of
 *    each level is computed once per band, plus the levels*(levels-1) rows a
 *    band start needs and the column halo of `levels` on each side of a strip;
 *  - register tile (levels 1..6): a wave holds its output block grown by
 *    `levels` rows and columns and recomputes that halo.
 * Bit-identical to sten_jacobi5_f64 / _f32 (same arithmetic per point and
 * level, Section III-A). Needs 16-byte aligned u0/out/work and ld a multiple
 * of 2 (FP64) or 4 (FP32), an interior and T >= 1; returns
 * STEN_ERR_UNSUPPORTED otherwise (use the single-sweep entry points for those
 * grids). STEN_ERR_ARG for levels outside the chosen kernel's range. Other
 * errors as for sten_jacobi5_f64.
 */
sten_status sten_jacobi5_f64_tb(const double* u0, double* out, double* work, int64_t H, int64_t W, int64_t ld,
                                int32_t T, double c, int32_t levels, hipStream_t stream);
sten_status sten_jacobi5_f32_tb(const float* u0, float* out, float* work, int64_t H, int64_t W, int64_t ld,
                                int32_t T, float c, int32_t levels, hipStream_t stream);

/* Tuning hook for the temporally blocked kernels. variant: 0 built-in
 * (streaming), 1 register tile (it has launches of 1..6 sweeps; launches of
 * more sweeps, such as those of the plain calls' built-in schedule, still
 * take the streaming kernel, and sten_jacobi5_*_tb accepts levels up to 12,
 * FP64 up to 14, under either variant), 2 streaming. band: output rows per streaming
 * band (1..65536; 0 built-in: the tallest bands, in whole groups, that let
 * every resident wave slot hold one band). depth: rows the streaming kernel
 * loads ahead of the row it computes (0 or 4, the one depth built). Process-
 * wide; same bits for every setting. STEN_ERR_ARG for other values. */
sten_status sten_tune_tb(int32_t variant, int32_t band, int32_t depth);

/* Tuning hook: output rows per register tile of the temporally blocked
 * register-tile kernel (4, 8, 12 or 16; 0 restores the built-in 8). Same bits
 * for every value. */
sten_status sten_tune_tb_rows(int32_t rows);

/* Scalar slice fill (the listing's ring set-up, Section III-A): rows [r0, r1)
 * x columns [c0, c1) of an H x W FP64 grid get `value`. STEN_ERR_ARG when the
 * rectangle leaves the grid. */
sten_status sten_fill_rect_f64(double* grid, int64_t H, int64_t W, int64_t ld, int64_t r0, int64_t r1,
                               int64_t c0, int64_t c1, double value, hipStream_t stream);

/* Schedule hook for sten_jacobi5_f64 / _f32: sweeps per launch (1: one sweep
 * per launch, the paper's one kernel per iteration; 2..14: temporal blocking
 * with at most that many, FP32 calls taking at most 12; 0: built-in: while one
 * buffer is at most 128 MiB (the pair fits the Infinity Cache) 12 for FP64 and
 * 8 for FP32, above that 14 for FP64 and 12 for FP32). The T sweeps are split
 * evenly over ceil(T / levels) launches. Process-wide. Same bits for every
 * value. */
sten_status sten_tune_schedule(int32_t levels);

/* Tuning hook: output rows per workgroup tile of the sweep kernels (4, 8 or
 * 16; 0 restores the built-in choice). Process-wide; same bits for every
 * value. STEN_ERR_ARG for other values. */
sten_status sten_tune_sweep_rows(int32_t rows);

/* ------------------------------------------------------------------------ */
/* Cavity flow: blocked pressure iterations (Section V's second benchmark)  */
/* ------------------------------------------------------------------------ */
/*
 * nit Jacobi iterations of the lid-driven cavity flow's pressure equation,
 * each followed by its wall conditions, starting from p0 with source term b
 * (H x W FP64, row stride ld, device memory; the result goes to out). One
 * iteration maps p to q:
 *   q[i,j] = (cw * (p[i,j+1] + p[i,j-1]) + cn * (p[i+1,j] + p[i-1,j])) - cb * b[i,j]
 *            on rows 1..H-2, columns 1..W-2, evaluated in this order;
 *   q[i,W-1] = q[i,W-2], q[i,0] = q[i,1] on rows 1..H-2 (dp/dx = 0);
 *   q[0,:] = q[1,:] (dp/dy = 0, corners included); q[H-1,:] = 0 (the lid).
 * Up to `levels` iterations (1..12; 0 = 12) run per pass over HBM, the nit
 * iterations split as evenly as ceil(nit / levels) passes allow (50
 * iterations at the default: 5 passes of 10). The result is bit-identical to
 * applying the iteration nit times.
 * work: a second H x W buffer, needed when nit > levels (else may be NULL).
 * Errors: STEN_ERR_ARG (negative sizes or nit, ld < W, levels > 12);
 * STEN_ERR_PTR (NULL or non-device pointers); STEN_ERR_ALIAS (out or work
 * overlapping p0, b or each other); STEN_ERR_UNSUPPORTED for layouts the
 * blocked kernel does not take: H < 3, W < 128, W or ld odd, pointers not
 * 16-byte aligned, rows of 2^27 elements or more (the caller then runs the
 * iterations one at a time). nit = 0 copies p0 to out.
 */
sten_status sten_cavity_pressure_f64(const double* p0, const double* b, double* out, double* work, int64_t H,
                                     int64_t W, int64_t ld, int32_t nit, double cw, double cn, double cb,
                                     int32_t levels, hipStream_t stream);

/* Tuning hook of the blocked pressure kernel: rows per band (1..65536; 0
 * restores the built-in choice). Results unchanged. STEN_ERR_ARG otherwise. */
sten_status sten_tune_pressure(int32_t band);

/* ------------------------------------------------------------------------ */
/* Reduced-precision form: hi/lo encoding (extension; not in the paper)     */
/* ------------------------------------------------------------------------ */
/*
 * An FP64 grid x is stored as an FP32 plane hi = RN32(x) and an int16 plane
 * q with x ~= hi + q * delta(hi), delta(hi) = ulp32(hi) * 2^-16 (floored at
 * 2^-149): 6 bytes per point instead of 8, |x - decoded| <= 2^-40 |x|.
 * Layout of one encoded grid in a caller buffer `hilo` (256-byte aligned):
 * bytes [0, H*ld*4) hold the hi plane (row stride ld floats), followed, at
 * the next multiple of 256 bytes, by the q plane (row stride ld int16).
 * Each sweep decodes its inputs to FP32 pairs, sums them with error-free
 * FP32 transformations (double-word sums), multiplies by c as a double-word
 * product and re-encodes the result; FP64 is used only to encode and decode.
 */

/* Bytes of one encoded H x ld grid (hi plane + q plane, with alignment). */
size_t sten_hilo_bytes(int64_t H, int64_t ld);

/* Encode an FP64 grid. |x| must stay below the FP32 range (else the hi plane
 * holds inf). Bit-exact with the FP64 definition above (the one q value int16
 * cannot hold, +32768, is renormalised by stepping hi to the next FP32 value). */
sten_status sten_hilo_encode(const double* x, void* hilo, int64_t H, int64_t W, int64_t ld,
                             hipStream_t stream);

/* Decode to FP64 (exact: hi + q * delta is representable in FP64). */
sten_status sten_hilo_decode(const void* hilo, double* x, int64_t H, int64_t W, int64_t ld,
                             hipStream_t stream);

/*
 * T sweeps on encoded grids: src (never written) -> dst, with `work` as the
 * second ping-pong grid (needed when T >= 2). All three are encoded grids of
 * sten_hilo_bytes(H, ld) bytes each. The ring of dst (and work) is set from
 * src. Componentwise error vs the FP64 method on decode(src), J the T-sweep
 * map: |err| <= (T 2^-40 (1 + 2^-22) + T a)(1 + 2^-39)^T (|J| |x|), with
 * a = 17 * 2^-48 when c is a power of two and 20 * 2^-48 otherwise.
 */
sten_status sten_jacobi5_hilo(const void* src, void* dst, void* work,
                              int64_t H, int64_t W, int64_t ld, int32_t T, double c,
                              hipStream_t stream);

/* Bytes of `work` for sten_jacobi5_f64_hilo: two encoded grids. */
size_t sten_jacobi5_f64_hilo_work_bytes(int64_t H, int64_t ld);

/*
 * FP64 in, FP64 out through the hi/lo form: encode u0, T encoded sweeps,
 * decode into out. The ring of out is copied from u0 exactly; the interior
 * obeys the bound of sten_jacobi5_hilo (for T = 0 the interior is
 * decode(encode(u0)), within 2^-40 |u0|). work_bytes must be at least
 * sten_jacobi5_f64_hilo_work_bytes(H, ld) (else STEN_ERR_WORKSPACE); work
 * must be 256-byte aligned (else STEN_ERR_ARG).
 */
sten_status sten_jacobi5_f64_hilo(const double* u0, double* out, void* work, size_t work_bytes,
                                  int64_t H, int64_t W, int64_t ld, int32_t T, double c,
                                  hipStream_t stream);

/* Tuning hook: kernel variant of the hi/lo sweep. 1: register tiles of 4
 * rows x 4 points per lane; 2: 8 rows x 4 points; 3: 4 rows x 8 points; 4: 2
 * rows x 8 points; 5: row streaming over 16-row strips with loads 4 rows
 * ahead; 6: the same over 32-row strips; 7: 2 rows x 4 points; 8: 1 row x
 * 8 points; 9: 1 row x 16 points; 10: 3 rows x 8 points; 0: built-in choice
 * (4). All variants
 * give the same bits. STEN_ERR_ARG for other values. */
sten_status sten_tune_hilo_variant(int32_t variant);

/* ------------------------------------------------------------------------ */
/* Generated kernels for slice expressions (run-time code generation)        */
/* ------------------------------------------------------------------------ */

/*
 * The paper's backend generates one GPU kernel per AST, each thread computing
 * one element of the output slice, and compiles it at run time in every
 * process (Section III-C, code generation); consecutive assignments with the
 * same output shape and no dependence between them run as one kernel (node
 * fusion, Section III-B). These calls do that for FP64 slice expressions:
 * the library emits HIP source for a fused group, compiles it with hiprtc for
 * the current device, caches the code object per program and the kernel per
 * device, and launches one thread per two adjacent output elements of a row
 * (each operand pair one 16-byte load).
 *
 * Program text: one expression per output, separated by ';', each in postfix
 * form with blank-separated tokens:
 *   L<slot>,<di>,<dj>   input slot `slot` at row offset di, column offset dj
 *                        from the thread's output point
 *   C<number>            an FP64 constant (strtod syntax; hexadecimal floats
 *                        such as C0x1p-2 are exact)
 *   + - * /              binary operators; the left operand is pushed first
 *   N                    negation        Q   square (x * x)
 * Each operation rounds once to FP64 in program order (no fused multiply-add),
 * as NumPy evaluates the same expression element by element.
 */
typedef struct {
    const double* base;        /* element of the input aligned with output point (0, 0) */
    int64_t ld;                /* row stride in elements */
    int64_t row_lo, row_hi;    /* valid rows relative to base (inclusive); loads are checked against them */
    int64_t col_lo, col_hi;    /* valid columns relative to base (inclusive) */
} sten_expr_in;
typedef struct {
    double* base;              /* output point (0, 0) */
    int64_t ld;                /* row stride in elements (>= cols) */
} sten_expr_out;

/* Run a program over a rows x cols output region: output o gets expression o
 * at every point. Up to 16 input slots and 8 outputs. Checks before any
 * launch: program syntax and slot numbers (STEN_ERR_ARG, message in
 * sten_expr_log), every load inside its slot's extent (STEN_ERR_ARG), no
 * output overlapping an input extent or another output (STEN_ERR_ALIAS, the
 * paper's rule that an assignment may not read what it writes), device
 * pointers (STEN_ERR_PTR), rows < 2^31 and cols < 2^31 - 512 (STEN_ERR_ARG).
 * STEN_ERR_UNSUPPORTED if the run-time compiler fails (log in sten_expr_log).
 * rows or cols == 0: nothing to do. */
sten_status sten_expr_run(const char* program, const sten_expr_in* ins, int32_t nin, const sten_expr_out* outs,
                          int32_t nout, int64_t rows, int64_t cols, hipStream_t stream);

/* Host only (no GPU needed): the HIP source generated for `program`. Writes at
 * most cap bytes including the terminating NUL into buf; *len gets the full
 * length. STEN_ERR_ARG for an invalid program. */
sten_status sten_expr_source(const char* program, int32_t nin, int32_t nout, char* buf, size_t cap, size_t* len);

/* Host only: compile `program` for `arch` (NULL: "gfx950") with hiprtc and
 * cache the code object. STEN_ERR_UNSUPPORTED if compilation fails. */
sten_status sten_expr_compile(const char* program, int32_t nin, int32_t nout, const char* arch);

/* The last program or compiler message of the calling thread ("" if none). */
const char* sten_expr_log(void);

/* ------------------------------------------------------------------------ */
/* Batched form: many uneven grids in one persistent launch (extension)     */
/* ------------------------------------------------------------------------ */
/*
 * The paper runs one kernel per chare per iteration with many chares per GPU
 * (over-decomposition, Section III-C). Here a whole batch of independent FP32
 * grids, each iterated T times with the method, runs in one persistent
 * kernel: workgroups pull grids from an atomic queue (largest first) and run
 * all T sweeps of a grid with workgroup barriers only; grids whose ping-pong
 * pair fits the workgroup's LDS budget never touch HBM between load and store.
 * Results are bit-identical to sten_jacobi5_f32 on each grid.
 */

/* One grid of a batch: u0 [in], out [out], work [tmp, may be NULL when the
 * plan keeps the grid in LDS or T < 2], each H x W FP32 with row stride ld. */
typedef struct {
    const float* u0;
    float* out;
    float* work;
    int32_t H, W, ld, reserved;
} sten_inst;

/* Opaque host-side plan (owned by the caller; free with sten_batch_destroy). */
typedef struct sten_batch_plan_s* sten_batch_handle;

/* Device workspace bytes a plan of `count` grids needs (queue counter + descriptors). */
size_t sten_batch_workspace_bytes(int32_t count);

/*
 * Build a plan: validate every grid (STEN_ERR_ARG/PTR/ALIAS as for the plain
 * calls; a grid that sweeps in global memory with T >= 2 needs `work`), pick
 * the launch configuration (block size, LDS budget per workgroup, workgroups
 * per CU) from the tuning cache at tune_cache_path when it holds this batch's
 * key (else built-in defaults; the path may be NULL), classify and sort the
 * grids, and upload the sorted descriptors into dev_ws (device memory,
 * 256-byte aligned, >= sten_batch_workspace_bytes(count), else
 * STEN_ERR_WORKSPACE) with an async copy on `stream`. The plan keeps the
 * pointers: the buffers must stay valid while the plan is used.
 */
sten_status sten_batch_plan(const sten_inst* insts, int32_t count, int32_t T, float c,
                            const char* tune_cache_path, void* dev_ws, size_t ws_bytes,
                            sten_batch_handle* plan, hipStream_t stream);

/* Run the plan: a queue-reset kernel and the persistent kernel on `stream`.
 * Allocates nothing and issues no memset, so it can be captured in a HIP
 * graph. Runs of one plan must not overlap (they share the queue counter). */
sten_status sten_batch_run(sten_batch_handle plan, hipStream_t stream);

/* Autotuner: time every candidate configuration (block 256/512/1024 x LDS
 * budget 32/64/80/160 KiB within the device limit) on this batch, `reps`
 * runs each with HIP events (synchronises `stream`), each with the
 * register-resident mode on and off, keep the fastest in the
 * plan, report its time per run in *best_us (may be NULL) and append it to
 * the cache file (when the path is not NULL) for later sten_batch_plan calls.
 * Overwrites the grids' outputs. */
sten_status sten_batch_autotune(sten_batch_handle plan, const char* tune_cache_path, int32_t reps,
                                float* best_us, hipStream_t stream);

/* Set the launch configuration of a plan explicitly (block 64..1024, a power
 * of two; LDS budget in bytes, clamped to the device limit; workgroups per
 * CU 1..32) and re-classify its grids. STEN_ERR_ARG for values out of range. */
sten_status sten_batch_configure(sten_batch_handle plan, int32_t block, int32_t lds_bytes, int32_t wg_per_cu,
                                 hipStream_t stream);

/* Switch the register-resident mode on (1) or off (0) and re-classify the
 * grids. In that mode a workgroup holds the whole grid in registers (lanes
 * take columns, waves take row bands of at most 64 rows) and exchanges only
 * band-edge rows and wave-edge columns through LDS; it applies to grids with
 * ceil(W/64) <= waves per workgroup and enough bands for the rows. */
sten_status sten_batch_set_modes(sten_batch_handle plan, int32_t use_reg, hipStream_t stream);

/* Plan introspection: info[0..6] = block, LDS bytes, workgroups per CU, grid
 * size, grids kept in LDS, grids swept in global memory, grids only copied;
 * with n >= 9 also info[7] = grids held in registers, info[8] = register mode on. */
sten_status sten_batch_plan_info(sten_batch_handle plan, int32_t* info, int32_t n);

/* Free the host-side plan (device workspace stays the caller's). */
sten_status sten_batch_destroy(sten_batch_handle plan);

/* ------------------------------------------------------------------------ */
/* Adjoint: reverse mode of the FP32 method (extension; not in the paper)   */
/* ------------------------------------------------------------------------ */
/*
 * For L = sum(w * u_T), u_T the grid after T sweeps of the method from u0:
 * dL/du0 = (S^T)^T w, where one transposed sweep is, for every point n,
 *     (S^T g)[n] = [n on the ring] g[n] + c * (sum of g over n's interior neighbours)
 * (neighbour terms in the order N, S, W, E, exact zeros for missing ones,
 * FP32), and dL/dc = sum_k sum_{interior m} lambda_{k+1}[m] * nbrsum(u_k)[m]
 * with lambda_k = dL/du_k, which needs the forward states u_0..u_{T-1}.
 */

/* Doubles of `partials` the adjoint calls need for an H x W grid. */
size_t sten_adjoint_partials_len(int64_t H, int64_t W);

/* Forward FP32 method recording every state: states holds T+1 grids, state k
 * at states + k * H * ld (row stride ld); state 0 is a copy of u0, state k
 * the grid after k sweeps (bit-identical to sten_jacobi5_f32 with T = k). */
sten_status sten_jacobi5_f32_states(const float* u0, float* states, int64_t H, int64_t W, int64_t ld,
                                    int32_t T, float c, hipStream_t stream);

/* gin = dL/du0 for dL/du_T = gout: T transposed sweeps (work: second
 * ping-pong grid, needed when T >= 2). No two of gout, gin, work may overlap. */
sten_status sten_jacobi5_adjoint_f32(const float* gout, float* gin, float* work, int64_t H, int64_t W,
                                     int64_t ld, int32_t T, float c, hipStream_t stream);

/*
 * nsteps transposed sweeps over one segment of recorded states, for
 * checkpointed reverse passes: lam_in = dL/du_{k1}; states[s] = u_{k0+s}
 * (stride H * ld, s < nsteps, k1 = k0 + nsteps; may be NULL when dL/dc is not
 * wanted); lam_out = dL/du_{k0}. When partials (device, at least
 * sten_adjoint_partials_len(H, W) doubles) and states are given, each step
 * adds its dL/dc contribution into per-workgroup partial sums (FP64); reset
 * != 0 overwrites them first. Deterministic.
 */
sten_status sten_jacobi5_adjoint_f32_seg(const float* lam_in, const float* states, int32_t nsteps,
                                         float* lam_out, float* work, double* partials, int32_t reset,
                                         int64_t H, int64_t W, int64_t ld, float c, hipStream_t stream);

/* Tuning hook of the transposed steps without dL/dc: transposed steps per
 * launch of the several-step kernel (1..8; 0 restores the built-in choice).
 * Results unchanged. STEN_ERR_ARG otherwise. */
sten_status sten_tune_adjoint_levels(int32_t levels);

/* *out = sum of partials[0..n) in a fixed order (one workgroup). */
sten_status sten_reduce_f64(const double* partials, int64_t n, double* out, hipStream_t stream);

/*
 * For callers that cannot allocate device memory at call time (code under HIP
 * graph capture, tight serving loops): sten_jacobi5_adjoint_f32_seg with the
 * FP64 partial sums kept by the library, followed, when dLdc is not NULL, by
 * sten_reduce_f64 of those sums into *dLdc (device memory, one double).
 * Same bits as the two calls it replaces. The partial sums live in a static
 * per-device buffer of 2^20 doubles (8 MiB), held until the process ends;
 * grids needing more (sten_adjoint_partials_len(H, W) > 2^20) are rejected
 * with STEN_ERR_WORKSPACE. The buffer keeps the last call's sums: reset != 0
 * clears them (a fill kernel, no memset), reset == 0 adds this segment to
 * them, so a checkpointed reverse pass calls it once per segment, the first
 * with reset set, and *dLdc holds the running total after each call. All
 * calls on one device share the buffer: calls that overlap on one device
 * (other threads or streams) race. The lambda ping-pong grid `work` is the
 * caller's, as for sten_jacobi5_adjoint_f32_seg. Allocates nothing.
 */
sten_status sten_jacobi5_adjoint_f32_seg_noalloc(const float* lam_in, const float* states, int32_t nsteps,
                                                 float* lam_out, float* work, int32_t reset, double* dLdc,
                                                 int64_t H, int64_t W, int64_t ld, float c, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Tiled execution on one GPU (chares with ghost exchange)                   */
/* ------------------------------------------------------------------------ */
/*
 * The paper's data layout and DAG execution (Section III-C): an H x W FP64
 * grid split into pr x pc tiles, each with its owned block, a ghost frame of
 * depth g (1 is the ghost depth of the five-point stencil) and two buffers.
 * Before a sweep reads an array, its ghosts are refreshed when its local
 * generation epoch differs from its ghost epoch, by exchange kernels on the
 * communication stream, ordered against the compute stream by a compute event
 * and a communication event. A frame of depth g > 1 lets every tile run up to
 * g sweeps between exchanges; its exchange also carries the g x g corner
 * blocks between diagonal neighbours. Results are bit-identical to
 * sten_jacobi5_f64 on the whole grid for any tiling, depth and mode.
 */
typedef struct sten_tiled_s* sten_tiled_handle;

/* Exchange modes. PACKED: the paper's scheme, a pack kernel into one send
 * buffer per neighbour (in the workspace) and an unpack kernel into the ghost
 * frames. DIRECT: one kernel copies each neighbour's boundary block straight
 * into the ghost frame (no send buffers). */
typedef enum { STEN_TILED_PACKED = 0, STEN_TILED_DIRECT = 1 } sten_tiled_mode;

/* Device workspace bytes for a tiling with ghost depth 1, packed mode (0 when
 * the tiling is invalid: H, W, pr, pc < 1, more tiles than rows/columns, or
 * more than 65536 tiles in all). */
size_t sten_tiled_workspace_bytes(int64_t H, int64_t W, int32_t pr, int32_t pc);

/* Device workspace bytes for a tiling with ghost depth `ghost` (1..12) and
 * exchange mode `mode`; 0 when the tiling is invalid: as above, or a tile
 * thinner than `ghost` across an edge it shares with a neighbour, or an
 * unknown mode, or (ghost > 1) rows of 2^27 elements or more. */
size_t sten_tiled_workspace_bytes_ex(int64_t H, int64_t W, int32_t pr, int32_t pc, int32_t ghost, int32_t mode);

/* Create the tiling inside dev_ws (device memory, 256-byte aligned, at least
 * sten_tiled_workspace_bytes). Ghost depth 1, packed mode. Tile (a, b) owns
 * rows [a H/pr, (a+1) H/pr) and columns [b W/pc, (b+1) W/pc) (integer
 * division). Host-side handle. */
sten_status sten_tiled_create(int64_t H, int64_t W, int32_t pr, int32_t pc, void* dev_ws, size_t ws_bytes,
                              sten_tiled_handle* out);

/* As sten_tiled_create with ghost depth `ghost` (1..12) and exchange mode
 * `mode`: sten_tiled_run then exchanges once per at most `ghost` sweeps.
 * STEN_ERR_ARG for an invalid tiling (see sten_tiled_workspace_bytes_ex),
 * STEN_ERR_WORKSPACE when ws_bytes is too small. */
sten_status sten_tiled_create_ex(int64_t H, int64_t W, int32_t pr, int32_t pc, int32_t ghost, int32_t mode,
                                 void* dev_ws, size_t ws_bytes, sten_tiled_handle* out);

/* Host-only check of a tiling's plan (no HIP call): lays the workspace out at a
 * stand-in address and checks that every exchange copy, owned block and sweep
 * view lies inside its buffer, that each message matches its ghost block, and
 * that views are 16-byte aligned. info[0..3] = tiles, messages per exchange,
 * exchange kernel launches, workspace bytes (n >= 4). STEN_OK when the plan
 * passes; STEN_ERR_ARG for an invalid tiling; STEN_ERR_UNSUPPORTED if a check
 * fails (sten_tiled_create_ex runs the same check and refuses such a plan). */
sten_status sten_tiled_plan_check(int64_t H, int64_t W, int32_t pr, int32_t pc, int32_t ghost, int32_t mode,
                                  int64_t* info, int32_t n);

/* Load a grid u (row stride ld) into both buffers of every tile; ghosts become
 * stale (epochs advance). */
sten_status sten_tiled_scatter(sten_tiled_handle t, const double* u, int64_t ld, hipStream_t stream);

/* T sweeps with coefficient c, in ceil(T / g) chunks of at most g sweeps (split
 * as evenly as that count allows): per chunk, a ghost exchange of the array
 * being read (when stale) on `comm`, then on `compute` either one sweep kernel
 * per tile (chunks of one sweep) or one launch of the streaming blocked kernel
 * over all tiles (per 32 tiles). The streams may be the same (then no events
 * are recorded). */
sten_status sten_tiled_run(sten_tiled_handle t, int32_t T, double c, hipStream_t compute, hipStream_t comm);

/* Refresh the current array's ghosts if stale (a second call in a row is skipped). */
sten_status sten_tiled_exchange(sten_tiled_handle t, hipStream_t compute, hipStream_t comm);

/* Write the current state of every tile's owned block into u (row stride ld). */
sten_status sten_tiled_gather(sten_tiled_handle t, double* u, int64_t ld, hipStream_t stream);

/* stats[0..4] = tiles, exchanges performed, exchanges skipped (epochs equal),
 * sweep kernel launches, messages per exchange; stats[5] = ghost depth and
 * stats[6] = mode when n >= 7. */
sten_status sten_tiled_stats(sten_tiled_handle t, int64_t* stats, int32_t n);

/* Free the host-side handle (the workspace stays the caller's). */
sten_status sten_tiled_destroy(sten_tiled_handle t);

/* ------------------------------------------------------------------------ */
/* General star stencils with node fusion                                    */
/* ------------------------------------------------------------------------ */
/*
 * The class of slice expressions the paper's backend turns into kernels
 * (Section III-C): a constant-coefficient star stencil of radius R (1..4),
 *     out[i,j] = c0*A[i,j] + sum_{k=1..R} (cn[k-1]*A[i-k,j] + cs[k-1]*A[i+k,j]
 *                                         + cw[k-1]*A[i,j-k] + ce[k-1]*A[i,j+k])
 * evaluated left to right in that order, each product rounded then added (no
 * fused multiply-add), on points at least R away from every edge; the frame of
 * width R is not written. Ghost depth = R. Bit-identical to that expression
 * evaluated in FP64.
 */
typedef struct {
    int32_t radius;   /* 1..4 */
    int32_t reserved;
    double c0;
    double cn[4], cs[4], cw[4], ce[4];  /* entries past the radius are ignored */
} sten_star_coef;

/* Node fusion (Section III-B): nout (1..4) stencils of the same radius applied
 * to the same input in one kernel, which reads `in` once. outs: host array of
 * nout device pointers (grids of the same H, W, ld). STEN_ERR_ARG when radii
 * differ or are out of range; STEN_ERR_ALIAS when any two grids overlap. */
sten_status sten_star_f64(const double* in, double* const* outs, const sten_star_coef* coefs, int32_t nout,
                          int64_t H, int64_t W, int64_t ld, hipStream_t stream);

/* T applications of one star stencil with a ping-pong swap: out (and work,
 * needed when T >= 2) start as copies of u0, so the frame stays u0's. */
sten_status sten_star_iterate_f64(const double* u0, double* out, double* work, const sten_star_coef* coef,
                                  int64_t H, int64_t W, int64_t ld, int32_t T, hipStream_t stream);

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
