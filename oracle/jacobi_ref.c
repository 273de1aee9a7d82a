/*
 * Plain C + OpenMP twin of the CPU oracle for the 2-D five-point Jacobi sweep.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code with
 * the GPU library.
 *
 * It computes what the listing of the Laplace solver (Section III-A) computes:
 * both buffers start as copies of u0 (so both carry u0's boundary ring); each
 * sweep writes every interior point of one buffer as
 *     c * (((up + down) + left) + right)
 * from the other buffer, in that order, then the buffers swap. The result is
 * the last-written buffer, copied to `out`. Rows are split among OpenMP
 * threads; each point is computed the same way whatever the thread count, so
 * the result is bit-identical to the NumPy oracle. Build with
 * -ffp-contract=off so that no multiply-add is fused.
 */
#include <stdint.h>
#include <string.h>
#include <omp.h>

static void copy_grid_f64(double* dst, const double* src, int64_t n) {
    memcpy(dst, src, (size_t)n * sizeof(double));
}

static void copy_grid_f32(float* dst, const float* src, int64_t n) {
    memcpy(dst, src, (size_t)n * sizeof(float));
}

/* u0, out, work: H*W contiguous row-major grids (row stride W). */
int oracle_jacobi5_f64(const double* u0, double* out, double* work,
                       int64_t H, int64_t W, int32_t T, double c, int32_t nthreads) {
    if (H < 0 || W < 0 || T < 0) return -1;
    int64_t n = H * W;
    double* a = out;
    double* b = work;
    copy_grid_f64(a, u0, n);
    copy_grid_f64(b, u0, n);
    if (H < 3 || W < 3) return 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    for (int32_t t = 0; t < T; ++t) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 1; i < H - 1; ++i) {
            for (int64_t j = 1; j < W - 1; ++j) {
                double up = a[(i - 1) * W + j];
                double down = a[(i + 1) * W + j];
                double left = a[i * W + j - 1];
                double right = a[i * W + j + 1];
                b[i * W + j] = c * (((up + down) + left) + right);
            }
        }
        double* tmp = a; a = b; b = tmp;
    }
    if (a != out) copy_grid_f64(out, a, n);
    return 0;
}

int oracle_jacobi5_f32(const float* u0, float* out, float* work,
                       int64_t H, int64_t W, int32_t T, float c, int32_t nthreads) {
    if (H < 0 || W < 0 || T < 0) return -1;
    int64_t n = H * W;
    float* a = out;
    float* b = work;
    copy_grid_f32(a, u0, n);
    copy_grid_f32(b, u0, n);
    if (H < 3 || W < 3) return 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    for (int32_t t = 0; t < T; ++t) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 1; i < H - 1; ++i) {
            for (int64_t j = 1; j < W - 1; ++j) {
                float up = a[(i - 1) * W + j];
                float down = a[(i + 1) * W + j];
                float left = a[i * W + j - 1];
                float right = a[i * W + j + 1];
                b[i * W + j] = c * (((up + down) + left) + right);
            }
        }
        float* tmp = a; a = b; b = tmp;
    }
    if (a != out) copy_grid_f32(out, a, n);
    return 0;
}

/* Number of threads an OpenMP parallel region would use after the request. */
int oracle_threads(int32_t nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int used = 1;
    #pragma omp parallel
    {
        #pragma omp single
        used = omp_get_num_threads();
    }
    return used;
}
