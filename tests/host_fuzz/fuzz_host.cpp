// Seeded fuzz driver for libsten's host-side parsers and planners, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (the
// library sources are compiled host-only; no GPU is needed or used).
//
// Exercised: the expression-program parser and source generator
// (sten_expr_source), the tiling planner and its bounds check
// (sten_tiled_plan_check, sten_tiled_workspace_bytes_ex), the batch plan's
// argument validation (sten_batch_plan with host pointers stops at the device
// pointer check) and the workspace queries. Every call must return one of the
// documented status codes, and the results must agree with each other.
//
// Usage: fuzz_host <seed> <iterations>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "sten.h"

namespace sten {
// Kernel launchers of the GPU sources, which this host-only build leaves out;
// the paths fuzzed here never launch.
template <typename T>
struct GridView;
bool launch_stream_grids_f64(const GridView<double>*, int, double, int, hipStream_t) {
    std::fprintf(stderr, "unexpected launch\n");
    std::abort();
}
struct GridMirror;
bool launch_sweep_grids_f64(const GridView<double>*, int, double, hipStream_t, const GridMirror*) {
    std::fprintf(stderr, "unexpected launch\n");
    std::abort();
}
void launch_sweep_f64_internal(const double*, double*, int, int, int64_t, double, hipStream_t) {
    std::fprintf(stderr, "unexpected launch\n");
    std::abort();
}
}  // namespace sten

// The mixed form's workspace size lives in hilo.hip, also left out: the
// queries fuzzed here only need a deterministic value for it.
extern "C" size_t sten_jacobi5_f64_hilo_work_bytes(int64_t H, int64_t ld) { return (size_t)(H > 0 ? H : 0) * 16u + (size_t)(ld > 0 ? ld : 0); }

static int failures = 0;
#define EXPECT(cond, ...)                                  \
    do {                                                   \
        if (!(cond)) {                                     \
            std::fprintf(stderr, "FAIL %s: ", #cond);      \
            std::fprintf(stderr, __VA_ARGS__);             \
            std::fprintf(stderr, "\n");                    \
            ++failures;                                    \
        }                                                  \
    } while (0)

static bool is_status(int s) { return s <= 0 && s >= -6; }

// A random program: mostly well-formed postfix tokens, with random damage.
static std::string random_program(std::mt19937_64& rng, int nin, int nout) {
    std::uniform_int_distribution<int> u(0, 99);
    const char* ops[] = {"+", "-", "*", "/", "N", "Q"};
    std::string p;
    const int nexpr = std::max(1, nout + (u(rng) < 10 ? (u(rng) % 3) - 1 : 0));
    for (int e = 0; e < nexpr; ++e) {
        if (e) p += (u(rng) < 95) ? " ; " : ";;";
        int depth = 0;
        const int ntok = 1 + u(rng) % 40;
        for (int t = 0; t < ntok; ++t) {
            const int r = u(rng);
            if (r < 40) {
                const int slot = (u(rng) < 90) ? u(rng) % std::max(1, nin) : u(rng) - 50;
                p += "L" + std::to_string(slot) + "," + std::to_string(u(rng) % 9 - 4) + "," +
                     std::to_string(u(rng) % 9 - 4);
                ++depth;
            } else if (r < 55) {
                const char* consts[] = {"C0.25", "C-1e300", "C0x1p-2", "C1e-320", "Cnan", "Cinf", "C", "C1e999",
                                        "C0x", "C-0"};
                p += consts[u(rng) % 10];
                ++depth;
            } else if (r < 95) {
                const char* op = ops[u(rng) % 6];
                p += op;
                depth -= (op[0] == 'N' || op[0] == 'Q') ? 0 : 1;
            } else {
                const char* junk[] = {"L", "L1", "L1,", "L1,2", "L99999999999,0,0", "L0,2147483647,0", "X", "",
                                      "\t", "L0,-2147483648,5", "Cnan(", "L0,0,0,"};
                p += junk[u(rng) % 12];
            }
            p += ' ';
        }
        // usually close the expression so that it is valid
        while (depth > 1 && u(rng) < 90) {
            p += "+ ";
            --depth;
        }
    }
    if (u(rng) < 3) p.assign(70000 + u(rng) * 10, 'L');  // long garbage
    if (u(rng) < 3) {                                      // many tokens
        p.clear();
        for (int k = 0; k < 70000; ++k) p += (k == 0) ? "L0,0,0 " : "L0,0,0 + ";
    }
    return p;
}

static void fuzz_expr(std::mt19937_64& rng) {
    std::uniform_int_distribution<int> u(0, 99);
    const int nin = u(rng) % 20 - 2;
    const int nout = u(rng) % 11 - 1;
    const std::string prog = random_program(rng, nin, nout);
    const size_t caps[] = {0, 1, 7, 64, 4096, 1 << 20};
    const size_t cap = caps[u(rng) % 6];
    std::vector<char> buf(cap + 16, '#');
    size_t len = 12345;
    const int st = sten_expr_source(prog.c_str(), nin, nout, cap ? buf.data() : nullptr, cap, &len);
    EXPECT(is_status(st), "status %d", st);
    if (st == STEN_OK) {
        EXPECT(len > 0 && len < ((size_t)1 << 26), "length %zu", len);
        if (cap > 0) {
            const size_t written = std::min(len, cap - 1);
            EXPECT(buf[written] == '\0', "missing NUL at %zu", written);
            EXPECT(buf[cap] == '#', "wrote past cap %zu", cap);
        }
        EXPECT(nin >= 1 && nin <= 16 && nout >= 1 && nout <= 8, "accepted nin %d nout %d", nin, nout);
    }
    // a NULL program or length pointer is an argument error, not a crash
    EXPECT(sten_expr_source(nullptr, 1, 1, buf.data(), cap, &len) != STEN_OK, "NULL program accepted");
    const char* log = sten_expr_log();
    EXPECT(log != nullptr, "NULL log");
}

static void fuzz_tiled(std::mt19937_64& rng) {
    std::uniform_int_distribution<int> u(0, 99);
    auto pick64 = [&](void) -> int64_t {
        const int r = u(rng);
        if (r < 60) return 1 + u(rng) * 7 + u(rng);
        if (r < 75) return u(rng) % 5;
        if (r < 85) return -1 - u(rng);
        if (r < 95) return (int64_t)1 << (20 + u(rng) % 12);
        return ((int64_t)1 << 31) + u(rng) - 50;
    };
    const int64_t H = pick64(), W = pick64();
    const int32_t pr = u(rng) < 90 ? 1 + u(rng) % 9 : (u(rng) < 50 ? 0 : -1 - u(rng) % 3),
                  pc = u(rng) < 90 ? 1 + u(rng) % 9 : 1 << (u(rng) % 31);
    const int32_t ghost = u(rng) % 16 - 2, mode = u(rng) % 4 - 1;
    int64_t info[8] = {-7, -7, -7, -7, -7, -7, -7, -7};
    const int n = (u(rng) < 90) ? 4 + u(rng) % 5 : u(rng) % 4;
    const int st = sten_tiled_plan_check(H, W, pr, pc, ghost, mode, info, n);
    EXPECT(is_status(st), "plan_check status %d", st);
    const size_t ws = sten_tiled_workspace_bytes_ex(H, W, pr, pc, ghost, mode);
    if (st == STEN_OK) {
        EXPECT(n >= 4, "accepted n %d", n);
        EXPECT(info[0] == (int64_t)pr * pc, "tiles %lld for %d x %d", (long long)info[0], pr, pc);
        EXPECT((size_t)info[3] == ws && ws > 0, "workspace %lld vs %zu", (long long)info[3], ws);
        EXPECT(ghost >= 1 && ghost <= 12, "accepted ghost %d", ghost);
    }
    if (ws == 0) EXPECT(st != STEN_OK, "plan accepted with no workspace");
}

static void fuzz_workspace_queries(std::mt19937_64& rng) {
    std::uniform_int_distribution<int64_t> big(-5, ((int64_t)1 << 32));
    std::uniform_int_distribution<int> u(0, 99);
    const int op = u(rng) % 9 - 1;
    const int64_t H = u(rng) < 50 ? u(rng) : big(rng), W = u(rng) < 50 ? u(rng) : big(rng);
    const int32_t T = u(rng) < 80 ? u(rng) : (int32_t)(big(rng) - ((int64_t)1 << 31));
    const size_t b = sten_workspace_bytes(op, H, W, T);
    if (op < 0 || op > 5 || H < 0 || W < 0 || T < 0) EXPECT(b == STEN_WORKSPACE_INVALID, "op %d", op);
    (void)sten_batch_workspace_bytes((int32_t)(big(rng) - ((int64_t)1 << 31)));
}

static void fuzz_batch(std::mt19937_64& rng) {
    std::uniform_int_distribution<int> u(0, 99);
    const int count = u(rng) % 40;
    std::vector<sten_inst> insts(count);
    std::vector<float> host(64);
    for (auto& s : insts) {
        s.u0 = host.data();
        s.out = host.data() + 32;
        s.work = u(rng) < 50 ? nullptr : host.data() + 16;
        const int r = u(rng);
        s.H = r < 70 ? u(rng) * 3 : (r < 85 ? -u(rng) : INT32_MAX - u(rng));
        s.W = r < 70 ? u(rng) * 3 : (r < 85 ? INT32_MAX / 2 : -1);
        s.ld = (u(rng) < 80) ? s.W + u(rng) % 3 : s.W - 1;
        s.reserved = 0;
    }
    std::vector<char> ws(sten_batch_workspace_bytes(count) + 256);
    void* aligned = (void*)(((uintptr_t)ws.data() + 255) & ~(uintptr_t)255);
    sten_batch_handle h = nullptr;
    const int st = sten_batch_plan(count ? insts.data() : nullptr, count, u(rng) % 12 - 1, 0.25f, nullptr, aligned,
                                   ws.size() - 256, &h, nullptr);
    // host pointers are never device memory, so no plan can be made here
    EXPECT(st != STEN_OK && is_status(st) && h == nullptr, "batch status %d", st);
}

int main(int argc, char** argv) {
    const uint64_t seed = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 0;
    const int iters = argc > 2 ? std::atoi(argv[2]) : 2000;
    std::mt19937_64 rng(seed);
    for (int k = 0; k < iters; ++k) {
        fuzz_expr(rng);
        fuzz_tiled(rng);
        fuzz_workspace_queries(rng);
        if (k % 4 == 0) fuzz_batch(rng);
    }
    std::printf("fuzz_host seed %llu: %d iterations, %d failures\n", (unsigned long long)seed, iters, failures);
    return failures ? 1 : 0;
}
