// spec.cpp -- kernels specialised to one network structure and one formula.
//
// The generic persistent kernel interprets the network tables (reactants,
// state changes) and the compiled monitor program from device memory: every
// event pays scalar loads, loops over table entries and branches on entry
// kinds.  For small networks this interpretation costs more issue slots than
// the direct method's arithmetic itself.  Here the library writes the
// structure out as C++ constants (NetTab and MonProg values), compiles the
// same device code (ssa_core.h) against them with the HIP runtime compiler,
// and caches the resulting kernel per (device, structure).  Every table index
// then becomes an immediate and species counts live in registers; the
// arithmetic is unchanged, so results are identical to the generic kernel's.
//
// Rate constants, initial counts, seeds and stopping-rule parameters stay in
// the job table in device memory: one specialised kernel serves every rate
// set of a parameter sweep over the same network structure.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "smc_device.h"
#include "smc_internal.h"

namespace smc {

// Sources of the device headers, embedded at build time.
extern const char kEmbeddedDeviceHeader[];
extern const char kEmbeddedCoreHeader[];

namespace {

std::string fmt_double(double v)
{
    if (std::isinf(v)) return v > 0 ? "__builtin_inf()" : "(-__builtin_inf())";
    char buf[64];
    std::snprintf(buf, sizeof buf, "%a", v);
    return buf;
}

std::string fmt_i32(int32_t v)
{
    if (v == INT32_MIN) return "(-2147483647 - 1)";
    return std::to_string(v);
}

std::string fmt_i64(int64_t v)
{
    if (v == INT64_MIN) return "(-9223372036854775807LL - 1)";
    return std::to_string(v) + "LL";
}

std::string fmt_u64(uint64_t v)
{
    char buf[32];
    std::snprintf(buf, sizeof buf, "0x%" PRIx64 "ull", v);
    return buf;
}

struct Cache {
    std::mutex mu;
    std::map<std::pair<int, std::string>, hipFunction_t> fns;
};

Cache &cache()
{
    static Cache *c = new Cache();   // kept to process end with its modules
    return *c;
}

}  // namespace

// Small networks keep their counts in registers (StaticPolicy); wider ones,
// up to kSpecWideMaxS species and kSpecWideMaxM channels, in LDS
// (StaticWidePolicy).
bool spec_wide(int S, int M) { return S > kSpecMaxS || M > kSpecMaxM; }

bool spec_supported(int S, int M, const MonProg &mp)
{
    if (S < 1 || S > kSpecWideMaxS || M < 1 || M > kSpecWideMaxM) return false;
    if (mp.trace) return false;   // trace programs run on the generic kernel
    for (int q = 0; q < mp.n_preds; ++q)
        if (mp.preds[q].kind == PK_RPN) return false;
    return true;
}

std::string spec_source(int S, int M, const int32_t *reac, const uint32_t *chg, const MonProg &mp,
                        int waves_per_simd, bool iterative)
{
    std::string s;
    s.reserve(8192);
    s += "#include \"ssa_core.h\"\nnamespace smc {\nnamespace gen {\n";
    const std::string m = std::to_string(M);
    const bool wide = spec_wide(S, M);
    if (wide) {
        s += "constexpr ReacTab<" + m + "> make_wide()\n{\n    ReacTab<" + m + "> n{};\n";
        for (int i = 0; i < 2 * M; ++i)
            s += "    n.reac[" + std::to_string(i) + "] = " + fmt_i32(reac[i]) + ";\n";
        s += "    return n;\n}\n";
    } else {
        s += "constexpr NetTab<" + m + "> make_net()\n{\n    NetTab<" + m + "> n{};\n";
        for (int i = 0; i < 2 * M; ++i)
            s += "    n.reac[" + std::to_string(i) + "] = " + fmt_i32(reac[i]) + ";\n";
        for (int i = 0; i < 4 * M; ++i)
            s += "    n.chg[" + std::to_string(i) + "] = " + std::to_string(chg[i]) + "u;\n";
        s += "    return n;\n}\n";
    }
    s += "constexpr MonProg make_mon()\n{\n    MonProg m{};\n";
    s += "    m.n_preds = " + std::to_string(mp.n_preds) + ";\n";
    s += "    m.n_atoms = " + std::to_string(mp.n_atoms) + ";\n";
    s += "    m.n_props = " + std::to_string(mp.n_props) + ";\n";
    s += "    m.all_var = " + std::to_string(mp.all_var) + ";\n";
    for (int w = 0; w < 4; ++w) {
        s += "    m.topT[" + std::to_string(w) + "] = " + fmt_u64(mp.topT[w]) + ";\n";
        s += "    m.topF[" + std::to_string(w) + "] = " + fmt_u64(mp.topF[w]) + ";\n";
    }
    for (int a = 0; a < mp.n_atoms; ++a) {
        const Atom &A = mp.atoms[a];
        const std::string p = "    m.atoms[" + std::to_string(a) + "].";
        s += p + "kind = " + std::to_string(A.kind) + ";\n";
        s += p + "neg = " + std::to_string(A.neg) + ";\n";
        s += p + "p1 = " + std::to_string(A.p1) + ";\n";
        s += p + "p2 = " + std::to_string(A.p2) + ";\n";
        s += p + "p3 = " + std::to_string(A.p3) + ";\n";
        s += p + "slot = " + std::to_string(A.slot) + ";\n";
        s += p + "lo = " + fmt_double(A.lo) + ";\n";
        s += p + "hi = " + fmt_double(A.hi) + ";\n";
        s += p + "hi2 = " + fmt_double(A.hi2) + ";\n";
        s += p + "lo2 = " + fmt_double(A.lo2) + ";\n";
    }
    for (int q = 0; q < mp.n_props; ++q) {
        const Prop &P = mp.props[q];
        const std::string p = "    m.props[" + std::to_string(q) + "].";
        s += p + "off = " + std::to_string(P.off) + ";\n";
        s += p + "cnt = " + std::to_string(P.cnt) + ";\n";
        s += p + "table = " + std::to_string(P.table) + "u;\n";
    }
    for (int q = 0; q < mp.n_preds; ++q) {
        const Pred &P = mp.preds[q];
        const std::string p = "    m.preds[" + std::to_string(q) + "].";
        s += p + "kind = " + std::to_string(P.kind) + ";\n";
        s += p + "op = " + std::to_string(P.op) + ";\n";
        s += p + "var = " + std::to_string(P.var) + ";\n";
        s += p + "c32 = " + fmt_i32(P.c32) + ";\n";
        s += p + "lo32 = " + fmt_i32(P.lo32) + ";\n";
        s += p + "hi32 = " + fmt_i32(P.hi32) + ";\n";
        s += p + "neg = " + std::to_string(P.neg) + ";\n";
        s += p + "nterm = " + std::to_string(P.nterm) + ";\n";
        for (int k = 0; k < 4; ++k) {
            s += p + "vars[" + std::to_string(k) + "] = " + std::to_string(P.vars[k]) + ";\n";
            s += p + "w[" + std::to_string(k) + "] = " + fmt_i64(P.w[k]) + ";\n";
        }
        s += p + "c = " + fmt_i64(P.c) + ";\n";
    }
    s += "    m.horizon = " + fmt_double(mp.horizon) + ";\n";
    s += "    return m;\n}\n";
    s += "struct Spec {\n";
    s += "    static constexpr int S = " + std::to_string(S) + ";\n";
    s += "    static constexpr int M = " + m + ";\n";
    if (wide) s += "    static constexpr ReacTab<" + m + "> wide = make_wide();\n";
    else s += "    static constexpr NetTab<" + m + "> net = make_net();\n";
    s += "    static constexpr MonProg mon = make_mon();\n";
    s += "};\n}  // namespace gen\n}  // namespace smc\n";
    std::string attr = "__launch_bounds__(256)";
    if (waves_per_simd > 0)
        attr += " __attribute__((amdgpu_waves_per_eu(" + std::to_string(waves_per_simd) + ", 8)))";
    if (wide)
        s += "extern \"C\" __global__ " + attr + " void smc_spec_kernel(smc::KArgs A)\n{\n"
             "    extern __shared__ int32_t smc_lds[];\n"
             "    smc::persistent_body<smc::StaticWidePolicy<smc::gen::Spec>, " +
             std::string(iterative ? "true" : "false") + ">(A, smc_lds);\n}\n";
    else
        s += "extern \"C\" __global__ " + attr + " void smc_spec_kernel(smc::KArgs A)\n{\n"
             "    smc::persistent_body<smc::StaticPolicy<smc::gen::Spec>, " +
             std::string(iterative ? "true" : "false") + ">(A, nullptr);\n}\n";
    return s;
}

int spec_compile(const std::string &src, std::vector<char> &code, std::string &log)
{
    hiprtcProgram prog;
    const char *headers[] = {kEmbeddedDeviceHeader, kEmbeddedCoreHeader};
    const char *names[] = {"smc_device.h", "ssa_core.h"};
    if (hiprtcCreateProgram(&prog, src.c_str(), "smc_spec.hip", 2, headers, names) != HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return -1;
    }
    // Same code generation rules as the ahead-of-time kernels: no FP
    // contraction (the numeric contract), no packed FP32 instructions.
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t log_size = 0;
    if (hiprtcGetProgramLogSize(prog, &log_size) == HIPRTC_SUCCESS && log_size > 1) {
        log.assign(log_size, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
    }
    if (rc != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        if (log.empty()) log = hiprtcGetErrorString(rc);
        return -1;
    }
    size_t size = 0;
    hiprtcGetCodeSize(prog, &size);
    code.resize(size);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return 0;
}

int spec_kernel(int device, const std::string &src, hipFunction_t *fn, std::string &err)
{
    Cache &c = cache();
    std::lock_guard<std::mutex> lock(c.mu);
    const auto key = std::make_pair(device, src);
    auto it = c.fns.find(key);
    if (it != c.fns.end()) {
        *fn = it->second;
        return 0;
    }
    std::vector<char> code;
    std::string log;
    if (spec_compile(src, code, log) != 0) {
        err = "runtime compilation of the specialised kernel failed: " + log;
        return -1;
    }
    hipModule_t mod;
    hipError_t e = hipModuleLoadData(&mod, code.data());
    if (e != hipSuccess) {
        err = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
        return -1;
    }
    hipFunction_t f;
    e = hipModuleGetFunction(&f, mod, "smc_spec_kernel");
    if (e != hipSuccess) {
        err = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
        return -1;
    }
    c.fns.emplace(key, f);
    *fn = f;
    return 0;
}

}  // namespace smc
