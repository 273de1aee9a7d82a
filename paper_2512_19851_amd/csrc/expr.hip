// Run-time generated kernels for slice expressions: the paper's backend code
// generation (Section III-C) and node fusion (Section III-B) on gfx950.
//
// The frontend hands over one fused group of slice assignments with the same
// output shape as a small postfix program (grammar in sten.h). This file
// parses and validates it on the host, emits one HIP kernel for it (every
// operation rounds once, in program order, with no contraction into fused
// multiply-adds), compiles it with hiprtc for the device's architecture,
// caches the code object per program and the loaded function per device, and
// launches it.
//
// The paper's generator runs one thread per output element. Such kernels are
// bound by how many vector memory instructions they issue, not by their
// arithmetic or by HBM, so here a thread computes two adjacent elements of a
// row and moves each operand pair with one 16-byte load or store (8-byte
// aligned, which the hardware takes as one instruction); the last column of
// an odd-width row falls back to single elements.
//
// Nothing here touches the GPU until a launch: parsing, validation, source
// generation and compilation run on any host with ROCm, which is how the CPU
// tests exercise them.
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace sten {
namespace {

constexpr int kExprMaxIn = 16;
constexpr int kExprMaxOut = 8;
constexpr int kExprMaxTokens = 1 << 16;
constexpr int kExprMaxOffset = 1 << 20;
constexpr int kExprBlock = 256;
constexpr int kExprCols = 2;  // adjacent output columns per thread

// Kernel argument block; the generated source declares the same layout.
struct ExprArgs {
    const double* in[kExprMaxIn];
    int64_t ldi[kExprMaxIn];
    double* out[kExprMaxOut];
    int64_t ldo[kExprMaxOut];
    int32_t rows, cols, bpr, pad;
};

struct Token {
    enum Kind { LOAD, CONST, ADD, SUB, MUL, DIV, NEG, SQR } kind;
    int slot = 0, di = 0, dj = 0;
    double value = 0.0;
};

struct Program {
    std::vector<std::vector<Token>> outs;  // one postfix expression per output
};

thread_local std::string g_log;  // last parse or compile message of this thread

bool parse_int(const char*& p, long lo, long hi, int* v) {
    char* end = nullptr;
    long x = std::strtol(p, &end, 10);
    if (end == p || x < lo || x > hi) return false;
    *v = (int)x;
    p = end;
    return true;
}

// Parse and validate: slots < nin, exactly nout expressions, each leaving one
// value on the stack, finite constants, bounded offsets and length.
bool parse_program(const char* text, int nin, int nout, Program* prog) {
    prog->outs.assign(1, {});
    size_t ntok = 0;
    int depth = 0;
    const char* p = text;
    auto fail = [&](const char* why) {
        g_log = std::string("expression program: ") + why;
        return false;
    };
    while (true) {
        while (*p == ' ' || *p == '\t' || *p == '\n') ++p;
        if (*p == '\0' || *p == ';') {
            if (depth != 1) return fail("an expression must leave exactly one value");
            if (*p == '\0') break;
            ++p;
            prog->outs.emplace_back();
            depth = 0;
            continue;
        }
        if (++ntok > (size_t)kExprMaxTokens) return fail("too many tokens");
        Token t;
        const char c = *p++;
        switch (c) {
            case 'L':
                t.kind = Token::LOAD;
                if (!parse_int(p, 0, nin - 1, &t.slot) || *p++ != ',' ||
                    !parse_int(p, -kExprMaxOffset, kExprMaxOffset, &t.di) || *p++ != ',' ||
                    !parse_int(p, -kExprMaxOffset, kExprMaxOffset, &t.dj))
                    return fail("bad load token (L<slot>,<di>,<dj>)");
                ++depth;
                break;
            case 'C': {
                char* end = nullptr;
                t.kind = Token::CONST;
                t.value = std::strtod(p, &end);
                if (end == p || !std::isfinite(t.value)) return fail("bad constant");
                p = end;
                ++depth;
                break;
            }
            case '+': t.kind = Token::ADD; break;
            case '-': t.kind = Token::SUB; break;
            case '*': t.kind = Token::MUL; break;
            case '/': t.kind = Token::DIV; break;
            case 'N': t.kind = Token::NEG; break;
            case 'Q': t.kind = Token::SQR; break;
            default: return fail("unknown token");
        }
        if (t.kind == Token::ADD || t.kind == Token::SUB || t.kind == Token::MUL || t.kind == Token::DIV) {
            if (depth < 2) return fail("binary operator without two operands");
            --depth;
        } else if (t.kind == Token::NEG || t.kind == Token::SQR) {
            if (depth < 1) return fail("unary operator without an operand");
        }
        if (*p != '\0' && *p != ' ' && *p != '\t' && *p != '\n' && *p != ';') return fail("tokens must be separated");
        prog->outs.back().push_back(t);
    }
    if ((int)prog->outs.size() != nout) return fail("number of expressions differs from the number of outputs");
    return true;
}

std::string hex_double(double v) {
    char buf[64];
    std::snprintf(buf, sizeof(buf), "%a", v);
    return std::string("(") + buf + ")";
}

// The postfix program of one output as temporaries appended to `body`; a load
// token becomes the operand `load(slot, di, dj)` returns. Every operation gets
// its own temporary, so the compiled order is the program's order and each
// operation rounds once.
template <typename LoadName>
std::string emit_expression(const std::vector<Token>& e, LoadName load, int& tmp, std::string& body) {
    std::vector<std::string> st;
    for (const Token& t : e) {
        switch (t.kind) {
            case Token::LOAD: st.push_back(load(t.slot, t.di, t.dj)); break;
            case Token::CONST: st.push_back(hex_double(t.value)); break;
            case Token::NEG:
            case Token::SQR: {
                std::string x = st.back();
                st.pop_back();
                std::string name = "t" + std::to_string(tmp++);
                body += "    const double " + name + " = " + (t.kind == Token::NEG ? "-" + x : x + " * " + x) +
                        ";\n";
                st.push_back(name);
                break;
            }
            default: {
                std::string y = st.back();
                st.pop_back();
                std::string x = st.back();
                st.pop_back();
                const char* op = t.kind == Token::ADD ? " + " : t.kind == Token::SUB ? " - "
                               : t.kind == Token::MUL ? " * " : " / ";
                std::string name = "t" + std::to_string(tmp++);
                body += "    const double " + name + " = " + x + op + y + ";\n";
                st.push_back(name);
            }
        }
    }
    return st.back();
}

// One kernel for the whole group. A thread owns columns j and j + 1 of row i.
// With both inside the region, each distinct (slot, di, dj) is one 16-byte
// load of the pair at columns j + dj, j + dj + 1 (both inside the slot's
// checked extent), each element is evaluated from its half, and each output
// pair is one 16-byte store. A thread whose j is the region's last column
// loads and stores single values.
std::string generate_source(const Program& prog) {
    std::string s;
    s += "// generated by libsten for one fused group of slice assignments\n";
    s += "struct StenExprArgs { const double* in[" + std::to_string(kExprMaxIn) + "]; long long ldi[" +
         std::to_string(kExprMaxIn) + "]; double* out[" + std::to_string(kExprMaxOut) + "]; long long ldo[" +
         std::to_string(kExprMaxOut) + "]; int rows; int cols; int bpr; int pad; };\n";
    s += "typedef double sten_pair __attribute__((ext_vector_type(2), aligned(8)));\n";
    s += "extern \"C\" __global__ __launch_bounds__(" + std::to_string(kExprBlock) +
         ") void sten_expr_kernel(StenExprArgs a) {\n";
    s += "  const int b = (int)blockIdx.x;\n";
    s += "  const int i = b / a.bpr;\n";
    s += "  const int j = (b - i * a.bpr) * " + std::to_string(kExprBlock * kExprCols) + " + (int)threadIdx.x * " +
         std::to_string(kExprCols) + ";\n";
    s += "  if (j >= a.cols) return;\n";
    s += "  const long long r = i;\n";
    auto address = [](int slot, int di, int dj) {
        return "a.in[" + std::to_string(slot) + "] + (r + (" + std::to_string(di) + ")) * a.ldi[" +
               std::to_string(slot) + "] + (j + (" + std::to_string(dj) + "))";
    };
    int tmp = 0;
    // two elements
    {
        std::map<std::tuple<int, int, int>, std::string> pairs;
        std::string loads, body;
        auto pair_of = [&](int slot, int di, int dj) -> std::string {
            auto key = std::make_tuple(slot, di, dj);
            auto it = pairs.find(key);
            if (it == pairs.end()) {
                const std::string name = "p" + std::to_string(pairs.size());
                loads += "    const sten_pair " + name + " = *reinterpret_cast<const sten_pair*>(" +
                         address(slot, di, dj) + ");\n";
                it = pairs.emplace(key, name).first;
            }
            return it->second;
        };
        std::vector<std::string> res[2];
        for (int el = 0; el < 2; ++el)
            for (const auto& e : prog.outs)
                res[el].push_back(emit_expression(
                    e, [&](int slot, int di, int dj) { return pair_of(slot, di, dj) + (el == 0 ? ".x" : ".y"); },
                    tmp, body));
        s += "  if (j + 1 < a.cols) {\n" + loads + body;
        for (size_t o = 0; o < prog.outs.size(); ++o) {
            s += "    { sten_pair v; v.x = " + res[0][o] + "; v.y = " + res[1][o] + ";\n";
            s += "      *reinterpret_cast<sten_pair*>(a.out[" + std::to_string(o) + "] + r * a.ldo[" +
                 std::to_string(o) + "] + j) = v; }\n";
        }
        s += "    return;\n  }\n";
    }
    // the last column of an odd-width region
    {
        std::map<std::tuple<int, int, int>, std::string> vals;
        std::string loads, body;
        auto val_of = [&](int slot, int di, int dj) -> std::string {
            auto key = std::make_tuple(slot, di, dj);
            auto it = vals.find(key);
            if (it == vals.end()) {
                const std::string name = "l" + std::to_string(vals.size());
                loads += "    const double " + name + " = *(" + address(slot, di, dj) + ");\n";
                it = vals.emplace(key, name).first;
            }
            return it->second;
        };
        std::vector<std::string> res;
        for (const auto& e : prog.outs) res.push_back(emit_expression(e, val_of, tmp, body));
        s += "  {\n" + loads + body;
        for (size_t o = 0; o < prog.outs.size(); ++o)
            s += "    a.out[" + std::to_string(o) + "][r * a.ldo[" + std::to_string(o) + "] + j] = " + res[o] +
                 ";\n";
        s += "  }\n";
    }
    s += "}\n";
    return s;
}

std::mutex g_mu;
std::unordered_map<std::string, std::vector<char>> g_code;  // "arch\n" + source -> code object

// A validated program, its generated source and its kernel per device, cached by
// program text and slot counts, so a repeated launch neither parses nor
// generates again.
struct Prepared {
    Program prog;
    std::string src;
    std::map<int, hipFunction_t> fn;  // device -> loaded kernel (modules stay loaded)
};
std::unordered_map<std::string, std::unique_ptr<Prepared>> g_prepared;
constexpr size_t kMaxPrepared = 4096;

// Parse and generate once per (text, nin, nout). Caller holds g_mu.
Prepared* prepare_locked(const char* text, int nin, int nout) {
    std::string key = std::to_string(nin) + "," + std::to_string(nout) + ":" + text;
    auto it = g_prepared.find(key);
    if (it != g_prepared.end()) return it->second.get();
    auto p = std::make_unique<Prepared>();
    if (!parse_program(text, nin, nout, &p->prog)) return nullptr;
    p->src = generate_source(p->prog);
    if (g_prepared.size() >= kMaxPrepared) g_prepared.clear();  // bound the cache; loaded modules stay valid
    return g_prepared.emplace(std::move(key), std::move(p)).first->second.get();
}

// Compile (or fetch) the code object of `src` for `arch`. Caller holds g_mu.
sten_status compile_locked(const std::string& src, const std::string& arch, const std::vector<char>** code) {
    const std::string key = arch + "\n" + src;
    auto it = g_code.find(key);
    if (it != g_code.end()) {
        *code = &it->second;
        return STEN_OK;
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "sten_expr.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        g_log = "hiprtcCreateProgram failed";
        return STEN_ERR_UNSUPPORTED;
    }
    const std::string arch_opt = "--offload-arch=" + arch;
    const char* opts[] = {arch_opt.c_str(), "-O3", "-ffp-contract=off", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    size_t log_size = 0;
    g_log.clear();
    if (hiprtcGetProgramLogSize(prog, &log_size) == HIPRTC_SUCCESS && log_size > 1) {
        g_log.resize(log_size);
        hiprtcGetProgramLog(prog, &g_log[0]);
    }
    if (r != HIPRTC_SUCCESS) {
        g_log = std::string("hiprtc: ") + hiprtcGetErrorString(r) + "\n" + g_log;
        hiprtcDestroyProgram(&prog);
        return STEN_ERR_UNSUPPORTED;
    }
    size_t n = 0;
    std::vector<char> bin;
    if (hiprtcGetCodeSize(prog, &n) == HIPRTC_SUCCESS) {
        bin.resize(n);
        if (hiprtcGetCode(prog, bin.data()) != HIPRTC_SUCCESS) bin.clear();
    }
    hiprtcDestroyProgram(&prog);
    if (bin.empty()) {
        g_log = "hiprtc produced no code object";
        return STEN_ERR_UNSUPPORTED;
    }
    *code = &g_code.emplace(key, std::move(bin)).first->second;
    return STEN_OK;
}

std::string device_arch(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Byte range [lo, hi) covered by rows [r0, r1] x columns [c0, c1] of a grid with row stride ld.
void span_of(const double* base, int64_t ld, int64_t r0, int64_t r1, int64_t c0, int64_t c1, uintptr_t* lo,
             uintptr_t* hi) {
    *lo = (uintptr_t)(base + r0 * ld + c0);
    *hi = (uintptr_t)(base + r1 * ld + c1 + 1);
}

}  // namespace
}  // namespace sten

extern "C" {

const char* sten_expr_log(void) { return sten::g_log.c_str(); }

sten_status sten_expr_source(const char* program, int32_t nin, int32_t nout, char* buf, size_t cap, size_t* len) {
    using namespace sten;
    if (program == nullptr || nin < 1 || nin > kExprMaxIn || nout < 1 || nout > kExprMaxOut) return STEN_ERR_ARG;
    std::string src;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        Prepared* p = prepare_locked(program, nin, nout);
        if (p == nullptr) return STEN_ERR_ARG;
        src = p->src;
    }
    if (len != nullptr) *len = src.size();
    if (buf != nullptr && cap > 0) {
        const size_t n = std::min(cap - 1, src.size());
        std::memcpy(buf, src.data(), n);
        buf[n] = '\0';
    }
    return STEN_OK;
}

sten_status sten_expr_compile(const char* program, int32_t nin, int32_t nout, const char* arch) {
    using namespace sten;
    if (program == nullptr || nin < 1 || nin > kExprMaxIn || nout < 1 || nout > kExprMaxOut) return STEN_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    Prepared* p = prepare_locked(program, nin, nout);
    if (p == nullptr) return STEN_ERR_ARG;
    const std::vector<char>* code = nullptr;
    return compile_locked(p->src, arch != nullptr ? arch : "gfx950", &code);
}

sten_status sten_expr_run(const char* program, const sten_expr_in* ins, int32_t nin, const sten_expr_out* outs,
                          int32_t nout, int64_t rows, int64_t cols, hipStream_t stream) {
    using namespace sten;
    if (program == nullptr || ins == nullptr || outs == nullptr) return STEN_ERR_ARG;
    if (nin < 1 || nin > kExprMaxIn || nout < 1 || nout > kExprMaxOut || rows < 0 || cols < 0) return STEN_ERR_ARG;
    // the kernel forms a block's column indices in 32-bit arithmetic
    if (rows > INT32_MAX || cols > INT32_MAX - kExprBlock * kExprCols) return STEN_ERR_ARG;
    const int64_t bpr = (cols + kExprBlock * kExprCols - 1) / (kExprBlock * kExprCols);
    if (rows * bpr > INT32_MAX) return STEN_ERR_ARG;
    // One lock from parsing to the kernel lookup: the prepared program (owned by the cache) stays valid
    // while it is read. HIP calls made under it (pointer queries, compile, module load) call nothing back.
    hipFunction_t fn = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        Prepared* prep = prepare_locked(program, nin, nout);
        if (prep == nullptr) return STEN_ERR_ARG;
        if (rows == 0 || cols == 0) return STEN_OK;
        // every load stays inside its slot's declared extent
        for (const auto& e : prep->prog.outs)
            for (const Token& t : e)
                if (t.kind == Token::LOAD) {
                    const sten_expr_in& s = ins[t.slot];
                    if (t.di < s.row_lo || rows - 1 + t.di > s.row_hi || t.dj < s.col_lo ||
                        cols - 1 + t.dj > s.col_hi) {
                        g_log = "expression program: a load leaves its input's extent";
                        return STEN_ERR_ARG;
                    }
                }
        for (int k = 0; k < nin; ++k) {
            if (ins[k].ld < 1 || ins[k].row_lo > ins[k].row_hi || ins[k].col_lo > ins[k].col_hi) return STEN_ERR_ARG;
            if (ins[k].col_hi - ins[k].col_lo >= ins[k].ld) return STEN_ERR_ARG;
        }
        for (int o = 0; o < nout; ++o)
            if (outs[o].base == nullptr || outs[o].ld < cols) return STEN_ERR_ARG;
        // outputs overlap no input extent and no other output
        for (int o = 0; o < nout; ++o) {
            uintptr_t olo, ohi;
            span_of(outs[o].base, outs[o].ld, 0, rows - 1, 0, cols - 1, &olo, &ohi);
            for (int k = 0; k < nin; ++k) {
                uintptr_t ilo, ihi;
                span_of(ins[k].base, ins[k].ld, ins[k].row_lo, ins[k].row_hi, ins[k].col_lo, ins[k].col_hi, &ilo,
                        &ihi);
                if (olo < ihi && ilo < ohi) return STEN_ERR_ALIAS;
            }
            for (int q = 0; q < o; ++q) {
                uintptr_t qlo, qhi;
                span_of(outs[q].base, outs[q].ld, 0, rows - 1, 0, cols - 1, &qlo, &qhi);
                if (olo < qhi && qlo < ohi) return STEN_ERR_ALIAS;
            }
        }
        for (int k = 0; k < nin; ++k)
            if (!is_device_ptr(ins[k].base)) return STEN_ERR_PTR;
        for (int o = 0; o < nout; ++o)
            if (!is_device_ptr(outs[o].base)) return STEN_ERR_PTR;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e);
        auto it = prep->fn.find(dev);
        if (it != prep->fn.end()) {
            fn = it->second;
        } else {
            const std::string arch = device_arch(dev);
            if (arch.empty()) return hip_fail(hipGetLastError());
            const std::vector<char>* code = nullptr;
            sten_status st = compile_locked(prep->src, arch, &code);
            if (st != STEN_OK) return st;
            hipModule_t mod;
            e = hipModuleLoadData(&mod, code->data());
            if (e != hipSuccess) return hip_fail(e);
            e = hipModuleGetFunction(&fn, mod, "sten_expr_kernel");
            if (e != hipSuccess) return hip_fail(e);
            prep->fn.emplace(dev, fn);  // modules stay loaded for the process's lifetime
        }
    }
    ExprArgs a{};
    for (int k = 0; k < nin; ++k) {
        a.in[k] = ins[k].base;
        a.ldi[k] = ins[k].ld;
    }
    for (int o = 0; o < nout; ++o) {
        a.out[o] = outs[o].base;
        a.ldo[o] = outs[o].ld;
    }
    a.rows = (int32_t)rows;
    a.cols = (int32_t)cols;
    a.bpr = (int32_t)bpr;
    void* params[] = {&a};
    const hipError_t e = hipModuleLaunchKernel(fn, (unsigned)(rows * bpr), 1, 1, kExprBlock, 1, 1, 0, stream, params,
                                               nullptr);
    if (e != hipSuccess) return hip_fail(e);
    return STEN_OK;
}

}  // extern "C"
