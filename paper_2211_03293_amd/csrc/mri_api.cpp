// mri_api.cpp -- host side of libmri: argument validation, handles, the MRI
// slow-step driver, run-time specialization of the fast-stage kernels
// (hipRTC) and the batched work-queue plan.  See include/mri.h for the ABI.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <elf.h>
#include <sys/stat.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "mri.h"
#include "mri_surrogate.h"
#include "mri_dev.h"
#include "mri_internal.h"

// Embedded sources of the run-time compiled kernels (generated at build time).
extern const char mri_spec_kernels_src[];
extern const char mri_spec_abi_src[];
extern const char mri_math_src[];

thread_local std::string g_err;
// Cell counts and leading dimensions stay below 2^31 - 1024 so that a kernel's
// block index times block size (at most 1024) never leaves the int range.
constexpr long long kMaxCells = (1ll << 31) - 1024;

mri_status mri_fail(mri_status st, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

namespace {

constexpr double R_GAS = 8.314462618;  // J/(mol K)

#define fail mri_fail

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(MRI_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

std::atomic<int64_t> c_slow{0}, c_fast{0}, c_cells{0}, c_spec{0};

// Event pairs around fast-stage launches (benchmark timing).
struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    size_t used = 0;
};
Timing g_timing;

// Returns the pair to record around the next launch, or nullptr when off.
std::pair<hipEvent_t, hipEvent_t> *timing_slot()
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (!g_timing.on) return nullptr;
    if (g_timing.used == g_timing.pool.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return nullptr;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return nullptr;
        }
        g_timing.pool.emplace_back(a, b);
    }
    return &g_timing.pool[g_timing.used++];
}

bool finite_all(const double *p, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// One run-time compiled kernel: (block size, kind 0 RK4 / 1 Zonneveld /
// 2 batch work queue / 3 Heun / 4 Bogacki-Shampine, forcing terms).
struct SpecKernel {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    size_t code_bytes = 0;      // size of the code object it was loaded from
};

// Register / LDS tiling choices of a specialized kernel: the waves per SIMD its
// register allocation must allow, the exponential (2^(j/256) table in LDS or
// the polynomial), the scheduling window (rate evaluations per scheduling
// fence); 0 / -1 / 0 select the built-in heuristics of spec_kernels.inc.
struct SpecVariant {
    int wpe = 0;
    int exp_table = -1;
    int group = 0;
    bool operator==(const SpecVariant &o) const
    {
        return wpe == o.wpe && exp_table == o.exp_table && group == o.group;
    }
};

inline uint64_t spec_key(int wg, int kind, int np, const SpecVariant &v = SpecVariant())
{
    return (uint64_t)wg << 32 | (uint64_t)kind << 24 | (uint64_t)np << 20 |
           (uint64_t)(v.wpe & 7) << 16 | (uint64_t)((v.exp_table + 1) & 3) << 12 |
           (uint64_t)(v.group & 0xff);
}

std::string hexd(double v)
{
    char b[64];
    snprintf(b, sizeof b, "%a", v);
    return b;
}

}  // namespace

struct mri_mech {
    int kind = 0;     // 0 chemistry, 1 linear
    int S = 0, R = 0, n = 0;
    std::vector<double> sp, rx;
    std::vector<uint32_t> rxi;
    double T_ref = 0.0;
    std::vector<double> A;             // linear
    double *d_sp = nullptr, *d_rx = nullptr, *d_A = nullptr;
    uint32_t *d_rxi = nullptr;
    GenMech gm{};
    // run-time specialization
    std::mutex mu;
    std::string defs;                  // generated macro block
    std::map<uint64_t, SpecKernel> spec;    // by spec_key
    std::map<uint64_t, std::string> spec_fail;
    std::vector<char> last_code;       // code object of the last compilation
    ~mri_mech()
    {
        for (auto &kv : spec)
            if (kv.second.mod) (void)hipModuleUnload(kv.second.mod);
        if (d_sp) (void)hipFree(d_sp);
        if (d_rx) (void)hipFree(d_rx);
        if (d_rxi) (void)hipFree(d_rxi);
        if (d_A) (void)hipFree(d_A);
    }
};

struct mri_table {
    int s = 0, ng = 0;
    std::vector<double> c, gamma;
};

// ---------------------------------------------------------------------------
// Run-time specialization
// ---------------------------------------------------------------------------
// Literal tables of the specialized kernels (base-2 forms, see spec_kernels.inc):
// species (CFE = CF e^BR, WF, AR2 = AR log2 e, EA, CV); reactions
// (a, b, c, d, AP = e^(ln A'), beta, TH2 = theta' log2 e).
static std::string make_defs(const mri_mech &m)
{
    const double log2e = 1.4426950408889634074;
    std::ostringstream o;
    o << "#define NS " << m.S << "\n";
    o << "#define T_REF " << hexd(m.T_ref) << "\n";
    o << "#define MRI_SPECIES(X)";
    for (int k = 0; k < m.S; ++k) {
        const double *p = &m.sp[k * GEN_SP_STRIDE];
        o << " \\\n  X(" << k << ", " << hexd(p[0] * std::exp(p[3])) << ", " << hexd(p[1]) << ", "
          << hexd(p[2] * log2e) << ", " << hexd(p[4]) << ", " << hexd(p[5]) << ")";
    }
    o << "\n#define MRI_REACTIONS(X)";
    for (int j = 0; j < m.R; ++j) {
        const uint32_t id = m.rxi[j];
        o << " \\\n  X(" << (id & 255u) << ", " << ((id >> 8) & 255u) << ", "
          << ((id >> 16) & 255u) << ", " << (id >> 24) << ", " << hexd(std::exp(m.rx[3 * j]))
          << ", " << hexd(m.rx[3 * j + 1]) << ", " << hexd(m.rx[3 * j + 2] * log2e) << ")";
    }
    o << "\n";
    return o.str();
}

static std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::string a = prop.gcnArchName;
        const size_t colon = a.find(':');
        if (colon != std::string::npos) a = a.substr(0, colon);
        if (!a.empty()) return a;
    }
    return "gfx950";
}

static bool fixed_step(int method)
{
    return method == MRI_FAST_RK4 || method == MRI_FAST_HEUN || method == MRI_FAST_BS3 ||
           method == MRI_FAST_CK5;
}

// Cash-Karp's six-stage tableau, 5th-order solution (Cash and Karp 1990):
// nodes, weights and the full strictly lower-triangular stage matrix.
static ErkFull erk_full_ck5()
{
    ErkFull e{};
    e.s = 6;
    const double c[6] = {0.0, 1.0 / 5, 3.0 / 10, 3.0 / 5, 1.0, 7.0 / 8};
    const double b[6] = {37.0 / 378, 0.0, 250.0 / 621, 125.0 / 594, 0.0, 512.0 / 1771};
    const double a[6][5] = {{0, 0, 0, 0, 0},
                            {1.0 / 5, 0, 0, 0, 0},
                            {3.0 / 40, 9.0 / 40, 0, 0, 0},
                            {3.0 / 10, -9.0 / 10, 6.0 / 5, 0, 0},
                            {-11.0 / 54, 5.0 / 2, -70.0 / 27, 35.0 / 27, 0},
                            {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592,
                             253.0 / 4096}};
    for (int i = 0; i < 6; ++i) {
        e.c[i] = c[i];
        e.b[i] = b[i];
        for (int j = 0; j < 5; ++j) e.a[i][j] = a[i][j];
    }
    return e;
}

// Tableaus of the fixed-step methods in the form the kernels take (stage i's
// input uses only k_(i-1)): classic RK4; Heun (c = (0, 1), b = (1/2, 1/2),
// a21 = 1); Bogacki-Shampine's 3rd-order solution (c = (0, 1/2, 3/4),
// b = (2/9, 1/3, 4/9), a21 = 1/2, a32 = 3/4, a31 = 0).
static ErkCoef erk_coef(int method)
{
    ErkCoef e{};
    if (method == MRI_FAST_HEUN) {
        e.s = 2;
        e.c[1] = 1.0;
        e.b[0] = e.b[1] = 0.5;
        e.a[0] = 1.0;
    } else if (method == MRI_FAST_BS3) {
        e.s = 3;
        e.c[1] = 0.5, e.c[2] = 0.75;
        e.b[0] = 2.0 / 9.0, e.b[1] = 1.0 / 3.0, e.b[2] = 4.0 / 9.0;
        e.a[0] = 0.5, e.a[1] = 0.75;
    } else {
        e.s = 4;
        e.c[1] = e.c[2] = 0.5, e.c[3] = 1.0;
        e.b[0] = e.b[3] = 1.0 / 6.0, e.b[1] = e.b[2] = 1.0 / 3.0;
        e.a[0] = e.a[1] = 0.5, e.a[2] = 1.0;
    }
    return e;
}

// Run-time compiled kernel kind of a fast method: 0 RK4, 1 Zonneveld, 3 Heun,
// 4 Bogacki-Shampine, 5 Cash-Karp (2 is the batched work queue).
// run-time compiled kernel kind of the stiffness monitor (spec_kernels.inc)
constexpr int kStiffKind = 6;

static int spec_kind(int method)
{
    return method == MRI_FAST_RK4 ? 0
           : method == MRI_FAST_ZONNEVELD43 ? 1
           : method == MRI_FAST_HEUN ? 3
           : method == MRI_FAST_BS3 ? 4 : 5;
}

// Tableau macros of a full-tableau method for the run-time compiled kernel:
// nodes and weights selected by the stage index, the stage matrix by the
// (row, column) pair, all as literal constants (entries not listed are 0).
static std::string erk_full_defs(const ErkFull &e)
{
    auto sel = [&](const double *v) {
        std::string r = hexd(v[e.s - 1]);
        for (int i = e.s - 2; i >= 0; --i)
            r = "((j) == " + std::to_string(i) + " ? " + hexd(v[i]) + " : " + r + ")";
        return r;
    };
    std::string a = "0.0";
    for (int i = e.s - 1; i >= 1; --i)
        for (int j = i - 1; j >= 0; --j)
            if (e.a[i][j] != 0.0)
                a = "(((i) == " + std::to_string(i) + " && (j) == " + std::to_string(j) + ") ? " +
                    hexd(e.a[i][j]) + " : " + a + ")";
    return "#define MRI_ERK_S " + std::to_string(e.s) + "\n#define MRI_ERK_C(j) " + sel(e.c) +
           "\n#define MRI_ERK_B(j) " + sel(e.b) + "\n#define MRI_ERK_A(i, j) " + a + "\n";
}

// Tableau macros of a fixed-step method for the run-time compiled kernel:
// per-stage node, weight and next-input coefficient selected by the stage
// index with literal constants.
static std::string erk_defs(const ErkCoef &e)
{
    auto sel = [&](const double *v) {
        std::string r = hexd(v[e.s - 1]);
        for (int i = e.s - 2; i >= 0; --i)
            r = "((st) == " + std::to_string(i) + " ? " + hexd(v[i]) + " : " + r + ")";
        return r;
    };
    return "#define MRI_ERK_S " + std::to_string(e.s) + "\n#define MRI_ERK_COEF(st, cn, bw, ah) " +
           "const double cn = " + sel(e.c) + "; const double bw = " + sel(e.b) +
           "; const double ah = " + sel(e.a) + " * h;\n";
}

// Compile the specialized kernel (wg, kind, np); with load != 0 also load it
// on the current device.  Caller holds m->mu.
static mri_status spec_compile(mri_mech *m, int wg, int kind, int np, int load, SpecKernel *out,
                               const SpecVariant &var = SpecVariant())
{
    if (m->defs.empty()) m->defs = make_defs(*m);
    // Scheduling window (rate evaluations per sched barrier): small mechanisms
    // run two waves per SIMD, which hide latency, and prefer a tight window
    // (register pressure); large ones run one wave per SIMD and need the
    // instruction-level parallelism of a wider window (measured on MI355X:
    // 21 species 4.17 ms at 2 vs 4.34 ms at 8; 53 species 50.3 ms at 2 vs
    // 44.1 ms at 8, per 262,144-cell stage).
    int group = (m->S >= 40) ? 8 : 2;
    if (const char *g = std::getenv("MRI_SPEC_GROUP"))   // tuning knob
        group = std::max(1, std::atoi(g));
    if (var.group > 0) group = var.group;
    std::string tune = "#define MRI_GROUP " + std::to_string(group) + "\n";
    if (var.wpe > 0)
        tune += "#define MRI_WPE " + std::to_string(std::max(1, std::min(4, var.wpe))) + "\n";
    else if (const char *w = std::getenv("MRI_SPEC_WPE"))     // tuning knob: waves per SIMD
        tune += "#define MRI_WPE " + std::to_string(std::max(1, std::min(4, std::atoi(w)))) + "\n";
    if (var.exp_table >= 0)
        tune += std::string("#define MRI_EXP_TABLE ") + (var.exp_table ? "1" : "0") + "\n";
    else if (const char *e = std::getenv("MRI_SPEC_EXP_TABLE"))   // tuning knob: 0 / 1
        tune += std::string("#define MRI_EXP_TABLE ") + (std::atoi(e) ? "1" : "0") + "\n";
    if (kind == 3 || kind == 4) tune += erk_defs(erk_coef(kind == 3 ? MRI_FAST_HEUN : MRI_FAST_BS3));
    if (kind == 5) tune += erk_full_defs(erk_full_ck5());
    std::string src = m->defs + tune + "#define WG " + std::to_string(wg) + "\n#define MRI_KIND " +
                      std::to_string(kind) + "\n#define MRI_NP " + std::to_string(np) + "\n" +
                      mri_spec_kernels_src;
    if (const char *dir = std::getenv("MRI_SPEC_DUMP_DIR")) {
        // debugging aid: keep the generated source next to its headers
        const std::string base = std::string(dir) + "/mri_spec_w" + std::to_string(wg) + "_k" +
                                 std::to_string(kind) + "_p" + std::to_string(np);
        std::ofstream(base + ".hip") << src;
        std::ofstream(std::string(dir) + "/spec_abi.h") << mri_spec_abi_src;
        std::ofstream(std::string(dir) + "/mri_math.h") << mri_math_src;
    }
    const char *hdr_src[] = {mri_spec_abi_src, mri_math_src};
    const char *hdr_name[] = {"spec_abi.h", "mri_math.h"};
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "mri_spec.hip", 2, hdr_src, hdr_name) !=
        HIPRTC_SUCCESS)
        return fail(MRI_ECOMPILE, "hiprtcCreateProgram failed");
    const std::string arch = "--offload-arch=" + (load ? device_arch() : std::string("gfx950"));
    // Machine LICM would hoist every materialized 64-bit coefficient of the
    // straight-line rate code out of the substep loop and exhaust the register
    // file; rematerializing them next to their use is far cheaper.
    std::vector<std::string> extra;   // tuning knob: extra backend options, "-mllvm X" each
    if (const char *e = std::getenv("MRI_SPEC_LLVM_OPTS")) {
        std::istringstream in(e);
        for (std::string w; in >> w;) {
            extra.push_back("-mllvm");
            extra.push_back(w);
        }
    }
    std::vector<const char *> opts = {arch.c_str(), "-O3", "-std=c++17", "-ffp-contract=fast",
                                      "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                                      "-mllvm", "-disable-machine-licm"};
    for (const std::string &w : extra) opts.push_back(w.c_str());
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
    const uint64_t key = spec_key(wg, kind, np, var);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        if (log.size() > 800) log = log.substr(0, 800);
        m->spec_fail[key] = log;
        return fail(MRI_ECOMPILE, "hipRTC compilation failed: %s", log.c_str());
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    m->last_code.assign(cs, 0);
    hiprtcGetCode(prog, m->last_code.data());
    hiprtcDestroyProgram(&prog);
    if (const char *dir = std::getenv("MRI_SPEC_DUMP_DIR"))   // debugging aid
        std::ofstream(std::string(dir) + "/mri_spec_w" + std::to_string(wg) + "_k" +
                          std::to_string(kind) + "_p" + std::to_string(np) + ".co",
                      std::ios::binary)
            .write(m->last_code.data(), (std::streamsize)m->last_code.size());
    ++c_spec;
    if (!load) return MRI_OK;
    SpecKernel sk;
    sk.code_bytes = m->last_code.size();
    HIP_TRY(hipModuleLoadData(&sk.mod, m->last_code.data()));
    const hipError_t ge = hipModuleGetFunction(&sk.fn, sk.mod, "mri_spec_main");
    if (ge != hipSuccess) {
        (void)hipModuleUnload(sk.mod);
        return fail(MRI_EHIP, "hipModuleGetFunction failed: %s", hipGetErrorString(ge));
    }
    *out = sk;
    return MRI_OK;
}

static mri_status spec_get(mri_mech *m, int wg, int kind, int np, hipFunction_t *fn,
                           const SpecVariant &var = SpecVariant())
{
    std::lock_guard<std::mutex> lk(m->mu);
    const uint64_t key = spec_key(wg, kind, np, var);
    auto it = m->spec.find(key);
    if (it != m->spec.end()) {
        *fn = it->second.fn;
        return MRI_OK;
    }
    auto f = m->spec_fail.find(key);
    if (f != m->spec_fail.end())
        return fail(MRI_ECOMPILE, "specialization failed earlier: %s", f->second.c_str());
    SpecKernel sk;
    mri_status st = spec_compile(m, wg, kind, np, 1, &sk, var);
    if (st != MRI_OK) return st;
    m->spec.emplace(key, sk);
    *fn = sk.fn;
    return MRI_OK;
}

// Device copies of the mechanism are made on first device use, so handles can
// be created (and specialized kernels compiled) on a host without a GPU.
static mri_status ensure_device(mri_mech *m)
{
    std::lock_guard<std::mutex> lk(m->mu);
    if (m->kind == 1) {
        if (m->d_A) return MRI_OK;
        HIP_TRY(hipMalloc(&m->d_A, sizeof(double) * m->A.size()));
        HIP_TRY(hipMemcpy(m->d_A, m->A.data(), sizeof(double) * m->A.size(), hipMemcpyHostToDevice));
        return MRI_OK;
    }
    if (m->d_sp) return MRI_OK;
    // the generic kernels evaluate their exponentials in base 2: the exponent
    // coefficients (species a/R and b/R, reaction ln A' and theta') go to the
    // device multiplied by log2(e); beta multiplies log2(T) there instead of ln(T)
    const double log2e = 1.4426950408889634074;
    std::vector<double> sp2 = m->sp, rx2 = m->rx;
    for (int k = 0; k < m->S; ++k) {
        sp2[(size_t)k * GEN_SP_STRIDE + 2] *= log2e;
        sp2[(size_t)k * GEN_SP_STRIDE + 3] *= log2e;
    }
    for (int j = 0; j < m->R; ++j) {
        rx2[3 * (size_t)j] *= log2e;
        rx2[3 * (size_t)j + 2] *= log2e;
    }
    HIP_TRY(hipMalloc(&m->d_sp, sizeof(double) * sp2.size()));
    HIP_TRY(hipMalloc(&m->d_rx, sizeof(double) * rx2.size()));
    HIP_TRY(hipMalloc(&m->d_rxi, sizeof(uint32_t) * m->rxi.size()));
    HIP_TRY(hipMemcpy(m->d_sp, sp2.data(), sizeof(double) * sp2.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->d_rx, rx2.data(), sizeof(double) * rx2.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->d_rxi, m->rxi.data(), sizeof(uint32_t) * m->rxi.size(),
                      hipMemcpyHostToDevice));
    m->gm = GenMech{m->S, m->R, m->d_sp, m->d_rx, m->d_rxi, m->T_ref};
    return MRI_OK;
}

// ---------------------------------------------------------------------------
// Validation helpers
// ---------------------------------------------------------------------------
static mri_status check_opts(const mri_mech *m, const mri_fast_opts *o)
{
    if (!o) return fail(MRI_EINVAL, "opts is NULL");
    if (!fixed_step(o->method) && o->method != MRI_FAST_ZONNEVELD43)
        return fail(MRI_EINVAL, "unknown fast method %d", o->method);
    if (fixed_step(o->method) && o->n_sub < 1)
        return fail(MRI_EINVAL, "n_sub must be >= 1 (got %d)", o->n_sub);
    if (o->method == MRI_FAST_ZONNEVELD43) {
        if (!(o->rtol >= 0.0) || !(o->atol_Y > 0.0) || !(o->atol_T > 0.0) ||
            !std::isfinite(o->rtol) || !std::isfinite(o->atol_Y) || !std::isfinite(o->atol_T))
            return fail(MRI_EINVAL, "tolerances must be finite with atol > 0, rtol >= 0");
        if (o->max_steps < 1) return fail(MRI_EINVAL, "max_steps must be >= 1");
        if (m->kind == 1)
            return fail(MRI_EUNSUPPORTED, "linear test mode supports fixed-step methods only");
    }
    if (o->kernel < MRI_KERNEL_AUTO || o->kernel > MRI_KERNEL_SPECIALIZED)
        return fail(MRI_EINVAL, "unknown kernel selector %d", o->kernel);
    if (o->method == MRI_FAST_CK5 && m->kind == 0 && m->S > GEN_NMAX_SMALL)
        return fail(MRI_EUNSUPPORTED, "Cash-Karp 5 supports at most %d species", GEN_NMAX_SMALL);
    if (o->block_size != 0 && o->block_size != 64 && o->block_size != 128 &&
        o->block_size != 256)
        return fail(MRI_EINVAL, "block_size must be 0, 64, 128 or 256 (got %d)", o->block_size);
    if (!(o->stiff_limit >= 0.0) || !std::isfinite(o->stiff_limit))
        return fail(MRI_EINVAL, "stiff_limit must be finite and >= 0");
    return MRI_OK;
}

static int default_block(int kernel_kind) { return kernel_kind == MRI_KERNEL_GENERIC ? 64 : 128; }

// Launch one fast stage; `accumulate` ORs status and adds steps.
static mri_status fast_stage_launch(mri_mech *m, const mri_fast_opts *o, int n_cells, int ld,
                                  const double *yin, double *yout, int n_poly,
                                  const double *rho, double L, int32_t *status, int32_t *steps,
                                  int accumulate, hipStream_t s,
                                  const unsigned int *n_live = nullptr)
{
    if (n_cells == 0) return MRI_OK;
    mri_status dst = ensure_device(m);
    if (dst != MRI_OK) return dst;
    if (m->kind == 1) {
        if (n_live) return fail(MRI_EUNSUPPORTED, "device cell counts need a chemistry mechanism");
        if (o->method == MRI_FAST_CK5) {
            HIP_TRY(launch_lin_erk(m->n, m->d_A, erk_full_ck5(), n_cells, ld, yin, yout, n_poly,
                                   rho, L, o->n_sub, status, steps, accumulate, s));
        } else {
            HIP_TRY(launch_lin_rk4(m->n, m->d_A, erk_coef(o->method), n_cells, ld, yin, yout,
                                   n_poly, rho, L, o->n_sub, status, steps, accumulate, s));
        }
        ++c_fast;
        c_cells += n_cells;
        return MRI_OK;
    }
    // stiffness monitor at the stage start state: it writes (or ORs) the status
    // words and zeroes the step counts, and the stage then accumulates onto them
    if (o->stiff_limit > 0.0 && fixed_step(o->method) && (status || steps) && !n_live) {
        // the mechanism-specialized monitor where the stage runs specialized
        // kernels, else the generic one
        hipFunction_t sfn = nullptr;
        if (o->kernel != MRI_KERNEL_GENERIC && spec_get(m, 128, kStiffKind, 0, &sfn) == MRI_OK) {
            int nc = n_cells, ldv = ld, acc = accumulate, flag = MRI_CELL_STIFF;
            const double *yi = yin;
            double hh = L / o->n_sub, lim = o->stiff_limit;
            double *bnd = nullptr;
            int *stp = status, *sps = steps;
            void *args[] = {&nc, &ldv, &yi, &hh, &lim, &bnd, &stp, &sps, &acc, &flag};
            HIP_TRY(hipModuleLaunchKernel(sfn, (unsigned)((n_cells + 127) / 128), 1, 1, 128, 1, 1,
                                          0, s, args, nullptr));
        } else {
            HIP_TRY(launch_gen_stiff(m->gm, n_cells, ld, yin, L / o->n_sub, o->stiff_limit,
                                     nullptr, status, steps, accumulate, MRI_CELL_STIFF, s));
        }
        accumulate = 1;
    }
    int kind = o->kernel;
    hipFunction_t fn = nullptr;
    int wg = o->block_size;
    if (kind != MRI_KERNEL_GENERIC) {
        if (!wg) wg = default_block(MRI_KERNEL_SPECIALIZED);
        mri_status st = spec_get(m, wg, spec_kind(o->method), n_poly, &fn);
        if (st != MRI_OK) {
            if (kind == MRI_KERNEL_SPECIALIZED) return st;
            kind = MRI_KERNEL_GENERIC;
            wg = o->block_size;
        } else {
            kind = MRI_KERNEL_SPECIALIZED;
        }
    }
    if (kind == MRI_KERNEL_GENERIC) {
        if (!wg) wg = default_block(MRI_KERNEL_GENERIC);
        if (o->method == MRI_FAST_CK5) {
            // stage derivatives held in registers: at most GEN_NMAX_SMALL
            // species (checked with the options)
            HIP_TRY(launch_gen_erk(m->gm, erk_full_ck5(), wg, n_cells, ld, yin, yout, n_poly,
                                   rho, L, o->n_sub, status, steps, accumulate, n_live, s));
        } else if (fixed_step(o->method)) {
            HIP_TRY(launch_gen_rk4(m->gm, erk_coef(o->method), wg, n_cells, ld, yin, yout, n_poly,
                                   rho, L, o->n_sub, status, steps, accumulate, n_live, s));
        } else {
            ZvOpts z{o->rtol, o->atol_Y, o->atol_T, o->max_steps};
            HIP_TRY(launch_gen_zv(m->gm, wg, n_cells, ld, yin, yout, n_poly, rho, L, z, status,
                                  steps, accumulate, n_live, s));
        }
    } else {
        const unsigned grid = (unsigned)((n_cells + wg - 1) / wg);
        int nc = n_cells, ldv = ld, acc = accumulate;
        const double *yi = yin, *rh = rho;
        double *yo = yout;
        double Lv = L;
        int *stp = status, *sps = steps;
        const unsigned int *nl = n_live;
        if (fixed_step(o->method)) {
            int nsub = o->n_sub;
            void *args[] = {&nc, &ldv, &yi, &yo, &rh, &Lv, &nsub, &stp, &sps, &acc, &nl};
            HIP_TRY(hipModuleLaunchKernel(fn, grid, 1, 1, wg, 1, 1, 0, s, args,
                                          nullptr));
        } else {
            ZvOpts z{o->rtol, o->atol_Y, o->atol_T, o->max_steps};
            void *args[] = {&nc, &ldv, &yi, &yo, &rh, &Lv, &z, &stp, &sps, &acc, &nl};
            HIP_TRY(hipModuleLaunchKernel(fn, grid, 1, 1, wg, 1, 1, 0, s, args,
                                          nullptr));
        }
    }
    ++c_fast;
    c_cells += n_cells;
    return MRI_OK;
}

static mri_status fast_stage_impl(mri_mech *m, const mri_fast_opts *o, int n_cells, int ld,
                                  const double *yin, double *yout, int n_poly,
                                  const double *rho, double L, int32_t *status, int32_t *steps,
                                  int accumulate, hipStream_t s,
                                  const unsigned int *n_live = nullptr)
{
    if (n_cells == 0) return MRI_OK;
    auto *ev = timing_slot();
    if (ev) HIP_TRY(hipEventRecord(ev->first, s));
    mri_status st = fast_stage_launch(m, o, n_cells, ld, yin, yout, n_poly, rho, L, status, steps,
                                      accumulate, s, n_live);
    if (ev) HIP_TRY(hipEventRecord(ev->second, s));
    return st;
}

// ---------------------------------------------------------------------------
// Batched uneven sets
// ---------------------------------------------------------------------------
struct mri_batch_plan {
    mri_mech *mech = nullptr;
    mri_fast_opts opts{};
    int n_sets = 0;
    long long n_total = 0;
    std::vector<long long> off;
    long long *d_off = nullptr;
    double *d_L = nullptr;
    unsigned long long *d_counters = nullptr;   // [0] queue, [1] useful, [2] issued
    int wg = 0, n_blocks = 0;                   // tuned tile
    SpecVariant var;                            // tuned register / LDS tiling
    float tune_ms = 0.0f;                       // timed ms of the choice
    bool tuned = false, from_cache = false;
    struct Trial {
        int wg, blocks;
        SpecVariant var;
        float ms;
    };
    std::vector<Trial> tune_log;
    // captured launch (counter reset + persistent kernel), replayed while the
    // argument key is unchanged
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> graph_key;
    // releases whatever a partial creation or a run allocated
    ~mri_batch_plan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (d_off) (void)hipFree(d_off);
        if (d_L) (void)hipFree(d_L);
        if (d_counters) (void)hipFree(d_counters);
    }
};

mri_status mri_internal_fast_stage(mri_mech *m, const mri_fast_opts *o, int n_cells, int ld,
                                   const double *yin, double *yout, int n_poly, const double *rho,
                                   double L, int32_t *status, int32_t *steps, hipStream_t s,
                                   const unsigned int *n_live, int accumulate)
{
    mri_status st = check_opts(m, o);
    if (st != MRI_OK) return st;
    return fast_stage_impl(m, o, n_cells, ld, yin, yout, n_poly, rho, L, status, steps, accumulate,
                           s, n_live);
}

int mri_internal_state_width(const mri_mech *m) { return m ? m->n : -1; }
int mri_internal_is_chem(const mri_mech *m) { return m && m->kind == 0; }

// The Sec. 2.1 step after validation: F [s-1][n][ld] and rho [ng][n][ld] are
// device buffers the caller provides.  With timed = 0 no event is recorded
// around the fast stages (the path that must not create or allocate anything).
mri_status mri_internal_slow_step(mri_mech *m, const mri_table *t, const mri_fast_opts *opts,
                                  mri_slow_rhs f_slow, void *user, double t0, double H,
                                  int n_cells, int ld, double *y, double *F, double *rho,
                                  int32_t *status_out, int32_t *steps_out, int timed,
                                  hipStream_t s)
{
    const size_t vec = (size_t)m->n * ld;
    const int s_ = t->s, ng = t->ng;
    mri_stream_t stream = (mri_stream_t)s;
    mri_status st = MRI_OK;
    // step 1: Y_1 = y_n; F_1 = f^S(t_n, Y_1)
    int rc = f_slow(t0, y, F, n_cells, ld, user, stream);
    if (rc != 0) return fail(MRI_EINVAL, "slow RHS callback returned %d", rc);
    ++c_slow;
    for (int i = 1; i < s_; ++i) {
        const double dc = t->c[i] - t->c[i - 1];
        const double L = dc * H;
        // step 2a: forcing coefficients from F_j, j < i
        ForcingCoef coef{};
        for (int k = 0; k < ng; ++k)
            for (int j = 0; j < i; ++j) coef.c[k * 8 + j] = t->gamma[((size_t)k * s_ + i) * s_ + j] / dc;
        HIP_TRY(launch_forcing((long long)vec, ng, i, F, (long long)vec, coef, rho, s));
        // steps 2b-2c: fast IVP over the stage, in place
        st = timed ? fast_stage_impl(m, opts, n_cells, ld, y, y, ng, rho, L, status_out,
                                     steps_out, i > 1 ? 1 : 0, s)
                   : fast_stage_launch(m, opts, n_cells, ld, y, y, ng, rho, L, status_out,
                                       steps_out, i > 1 ? 1 : 0, s);
        if (st != MRI_OK) return st;
        if (i < s_ - 1) {
            rc = f_slow(t0 + t->c[i] * H, y, F + (size_t)i * vec, n_cells, ld, user, stream);
            if (rc != 0) return fail(MRI_EINVAL, "slow RHS callback returned %d", rc);
            ++c_slow;
        }
    }
    // step 3: y_(n+1) = Y_s (already in y)
    return MRI_OK;
}

// Whether a fast stage with these options would have to create device state
// first (copy the mechanism, compile or load a specialized kernel).
bool mri_internal_stage_needs_setup(mri_mech *m, const mri_fast_opts *o, int n_poly)
{
    std::lock_guard<std::mutex> lk(m->mu);
    if (m->kind == 1) return m->d_A == nullptr;
    if (!m->d_sp) return true;
    if (o->kernel == MRI_KERNEL_GENERIC) return false;
    if (o->stiff_limit > 0.0 && fixed_step(o->method)) {
        const uint64_t sk = spec_key(128, kStiffKind, 0);
        auto si = m->spec.find(sk);
        if ((si == m->spec.end() || !si->second.fn) &&
            !(o->kernel == MRI_KERNEL_AUTO && m->spec_fail.count(sk)))
            return true;
    }
    const int wg = o->block_size ? o->block_size : default_block(MRI_KERNEL_SPECIALIZED);
    const uint64_t key = spec_key(wg, spec_kind(o->method), n_poly);
    auto it = m->spec.find(key);
    if (it != m->spec.end() && it->second.fn) return false;
    // automatic selection falls back to the generic kernel after a failed compilation
    return !(o->kernel == MRI_KERNEL_AUTO && m->spec_fail.count(key));
}

mri_status mri_internal_check_slow_step(const mri_mech *m, const mri_table *t,
                                        const mri_fast_opts *opts, mri_slow_rhs f_slow,
                                        double t0, double H, int n_cells, int ld)
{
    if (!m || !t) return fail(MRI_EINVAL, "mech or table is NULL");
    mri_status st = check_opts(m, opts);
    if (st != MRI_OK) return st;
    if (!f_slow) return fail(MRI_EINVAL, "slow RHS callback is NULL");
    if (n_cells < 0 || ld < n_cells) return fail(MRI_EINVAL, "need 0 <= n_cells <= ld");
    if (ld > kMaxCells) return fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    if ((long long)ld * m->n > (1ll << 31) - 1)
        return fail(MRI_EINVAL, "n * ld exceeds 2^31 - 1 elements");
    if (!(H > 0.0) || !std::isfinite(H) || !std::isfinite(t0))
        return fail(MRI_EINVAL, "H must be positive and finite");
    return MRI_OK;
}

int mri_internal_table_stages(const mri_table *t) { return t ? t->s : 0; }
int mri_internal_table_terms(const mri_table *t) { return t ? t->ng : 0; }

extern "C" {

int mri_abi_version(void) { return MRI_ABI_VERSION; }

const char *mri_last_error(void) { return g_err.c_str(); }

void mri_get_counters(mri_counters *out)
{
    if (!out) return;
    out->slow_evals = c_slow.load();
    out->fast_stages = c_fast.load();
    out->cell_stages = c_cells.load();
    out->specializations = c_spec.load();
}

mri_status mri_timing_enable(int enable)
{
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.on = enable != 0;
    return MRI_OK;
}

mri_status mri_timing_read(double *fast_ms, int64_t *n_launches, int reset)
{
    if (!fast_ms || !n_launches) return fail(MRI_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g_timing.mu);
    double tot = 0.0;
    for (size_t i = 0; i < g_timing.used; ++i) {
        HIP_TRY(hipEventSynchronize(g_timing.pool[i].second));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, g_timing.pool[i].first, g_timing.pool[i].second));
        tot += ms;
    }
    *fast_ms = tot;
    *n_launches = (int64_t)g_timing.used;
    if (reset) g_timing.used = 0;
    return MRI_OK;
}

void mri_reset_counters(void)
{
    c_slow = 0;
    c_fast = 0;
    c_cells = 0;
    c_spec = 0;
}

mri_status mri_mech_create(const mri_mech_desc *d, mri_mech **out)
{
    if (!out) return fail(MRI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(MRI_EINVAL, "desc is NULL");
    const int S = d->n_species, R = d->n_reactions;
    if (S < 1 || S > 255) return fail(MRI_EINVAL, "n_species must be in [1, 255] (got %d)", S);
    if (R < 1) return fail(MRI_EINVAL, "n_reactions must be >= 1 (got %d)", R);
    if (!d->reactants || !d->products || !d->lnA || !d->beta || !d->theta || !d->g_a ||
        !d->g_b || !d->W || !d->cv)
        return fail(MRI_EINVAL, "a mechanism array is NULL");
    for (int j = 0; j < 2 * R; ++j)
        if (d->reactants[j] < 0 || d->reactants[j] >= S || d->products[j] < 0 ||
            d->products[j] >= S)
            return fail(MRI_EINVAL, "species index out of range in reaction %d", j / 2);
    if (!finite_all(d->lnA, R) || !finite_all(d->beta, R) || !finite_all(d->theta, R) ||
        !finite_all(d->g_a, S) || !finite_all(d->g_b, S) || !finite_all(d->W, S) ||
        !finite_all(d->cv, S))
        return fail(MRI_EINVAL, "non-finite mechanism coefficient");
    for (int k = 0; k < S; ++k)
        if (!(d->W[k] > 0.0) || !(d->cv[k] > 0.0))
            return fail(MRI_EINVAL, "W and cv must be positive (species %d)", k);
    if (!(d->rho > 0.0) || !std::isfinite(d->rho) || !std::isfinite(d->T_ref))
        return fail(MRI_EINVAL, "rho must be positive and T_ref finite");
    std::unique_ptr<mri_mech> m(new mri_mech);
    m->kind = 0;
    m->S = S;
    m->R = R;
    m->n = S + 1;
    m->T_ref = d->T_ref;
    const double rho_cgs = d->rho * 1e-3;
    m->sp.resize((size_t)GEN_SP_STRIDE * S);
    double zmax = 0.0;
    for (int k = 0; k < S; ++k) {
        const double Wg = d->W[k] * 1e3;
        double *p = &m->sp[(size_t)k * GEN_SP_STRIDE];
        p[0] = rho_cgs / Wg;
        p[1] = Wg / rho_cgs;
        p[2] = d->g_a[k] / R_GAS;
        p[3] = d->g_b[k] / R_GAS;
        p[4] = d->g_a[k] / d->W[k];
        p[5] = d->cv[k];
        zmax = std::max(zmax, std::fabs(p[2]) / 200.0 + std::fabs(p[3]));
    }
    // exp(g_k/(R T)) and products of two of them must stay finite down to 200 K
    if (zmax > 300.0)
        return fail(MRI_EUNSUPPORTED,
                    "|g_k|/(R T) reaches %.1f at T = 200 K; the factorized rate form needs <= 300",
                    zmax);
    m->rx.resize((size_t)3 * R);
    m->rxi.resize(R);
    for (int j = 0; j < R; ++j) {
        const int a = d->reactants[2 * j], b = d->reactants[2 * j + 1];
        const int c = d->products[2 * j], dd = d->products[2 * j + 1];
        const double *pa = &m->sp[(size_t)a * GEN_SP_STRIDE], *pb = &m->sp[(size_t)b * GEN_SP_STRIDE];
        m->rx[3 * j] = d->lnA[j] - (pa[3] + pb[3]);
        m->rx[3 * j + 1] = d->beta[j];
        m->rx[3 * j + 2] = d->theta[j] + (pa[2] + pb[2]);
        m->rxi[j] = (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)c << 16) | ((uint32_t)dd << 24);
        if (std::fabs(m->rx[3 * j]) > 700.0)
            return fail(MRI_EUNSUPPORTED,
                        "reaction %d: ln A - (g_b,a + g_b,b)/R = %.1f is outside +-700", j,
                        m->rx[3 * j]);
    }
    *out = m.release();
    return MRI_OK;
}

mri_status mri_mech_create_linear(int n, const double *A, mri_mech **out)
{
    if (!out) return fail(MRI_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 16) return fail(MRI_EINVAL, "linear mode needs 1 <= n <= 16 (got %d)", n);
    if (!A) return fail(MRI_EINVAL, "A is NULL");
    if (!finite_all(A, n * n)) return fail(MRI_EINVAL, "non-finite entry in A");
    std::unique_ptr<mri_mech> m(new mri_mech);
    m->kind = 1;
    m->n = n;
    m->A.assign(A, A + n * n);
    *out = m.release();
    return MRI_OK;
}

void mri_mech_destroy(mri_mech *m) { delete m; }

int mri_mech_state_width(const mri_mech *m) { return m ? m->n : -1; }

// FNV-1a (64 bit) over the bytes the GPU executes: the .text and .rodata
// sections of the ELF code object (machine code, kernel descriptors, constant
// tables).  The rest of the object carries a compilation-unit id that hipRTC
// derives from the source text, so comments would otherwise change the hash.
// Falls back to the whole object if the ELF headers do not parse.
static uint64_t code_hash_bytes(const std::vector<char> &co)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const char *p, size_t n) {
        for (size_t i = 0; i < n; ++i) {
            h ^= (uint64_t)(unsigned char)p[i];
            h *= 1099511628211ull;
        }
    };
    const size_t size = co.size();
    Elf64_Ehdr eh;
    bool ok = size >= sizeof(eh);
    if (ok) {
        std::memcpy(&eh, co.data(), sizeof(eh));
        ok = std::memcmp(eh.e_ident, ELFMAG, SELFMAG) == 0 && eh.e_ident[EI_CLASS] == ELFCLASS64 &&
             eh.e_shentsize == sizeof(Elf64_Shdr) && eh.e_shstrndx < eh.e_shnum &&
             eh.e_shoff <= size && (size - eh.e_shoff) / sizeof(Elf64_Shdr) >= eh.e_shnum;
    }
    int found = 0;
    if (ok) {
        auto shdr = [&](int i) {
            Elf64_Shdr sh;
            std::memcpy(&sh, co.data() + eh.e_shoff + (size_t)i * sizeof(Elf64_Shdr), sizeof(sh));
            return sh;
        };
        const Elf64_Shdr strs = shdr(eh.e_shstrndx);
        ok = strs.sh_offset <= size && strs.sh_size <= size - strs.sh_offset;
        for (int i = 0; ok && i < eh.e_shnum; ++i) {
            const Elf64_Shdr sh = shdr(i);
            if (sh.sh_name >= strs.sh_size || sh.sh_type == SHT_NOBITS) continue;
            const char *name = co.data() + strs.sh_offset + sh.sh_name;
            const size_t room = strs.sh_size - sh.sh_name;
            const bool text = strncmp(name, ".text", room) == 0;
            const bool ro = strncmp(name, ".rodata", room) == 0;
            if (!text && !ro) continue;
            if (sh.sh_offset > size || sh.sh_size > size - sh.sh_offset) {
                ok = false;
                break;
            }
            mix(name, text ? 5 : 7);
            mix(co.data() + sh.sh_offset, sh.sh_size);
            ++found;
        }
    }
    if (!ok || found == 0) {
        h = 1469598103934665603ull;
        mix(co.data(), size);
    }
    return h;
}

// Validation shared by the specialization entry points.
static mri_status check_spec_request(const mri_mech *m, int method, int n_poly, int block_size)
{
    if (!m) return fail(MRI_EINVAL, "mech is NULL");
    if (m->kind != 0) return fail(MRI_EUNSUPPORTED, "linear test mode has no specialization");
    if (block_size != 64 && block_size != 128 && block_size != 256)
        return fail(MRI_EINVAL, "block_size must be 64, 128 or 256");
    if (!fixed_step(method) && method != MRI_FAST_ZONNEVELD43)
        return fail(MRI_EINVAL, "unknown fast method %d", method);
    if (n_poly < 0 || n_poly > 4) return fail(MRI_EINVAL, "n_poly must be in [0, 4]");
    if (method == MRI_FAST_CK5 && m->S > GEN_NMAX_SMALL)
        return fail(MRI_EUNSUPPORTED, "Cash-Karp 5 supports at most %d species", GEN_NMAX_SMALL);
    return MRI_OK;
}

mri_status mri_mech_specialize_method(mri_mech *m, int method, int n_poly, int block_size,
                                      int load, size_t *code_bytes)
{
    mri_status cs = check_spec_request(m, method, n_poly, block_size);
    if (cs != MRI_OK) return cs;
    const int kind = spec_kind(method);
    if (load) {
        hipFunction_t fn = nullptr;
        mri_status st = spec_get(m, block_size, kind, n_poly, &fn);
        if (st != MRI_OK) return st;
        std::lock_guard<std::mutex> lk(m->mu);
        if (code_bytes) *code_bytes = m->spec.at(spec_key(block_size, kind, n_poly)).code_bytes;
        return MRI_OK;
    }
    std::lock_guard<std::mutex> lk(m->mu);
    SpecKernel unused;
    mri_status st = spec_compile(m, block_size, kind, n_poly, 0, &unused);
    if (st == MRI_OK && code_bytes) *code_bytes = m->last_code.size();
    return st;
}

mri_status mri_mech_specialize_monitor(mri_mech *m, int load, size_t *code_bytes)
{
    mri_status cs = check_spec_request(m, MRI_FAST_RK4, 0, 128);
    if (cs != MRI_OK) return cs;
    if (load) {
        hipFunction_t fn = nullptr;
        mri_status st = spec_get(m, 128, kStiffKind, 0, &fn);
        if (st != MRI_OK) return st;
        std::lock_guard<std::mutex> lk(m->mu);
        if (code_bytes) *code_bytes = m->spec.at(spec_key(128, kStiffKind, 0)).code_bytes;
        return MRI_OK;
    }
    std::lock_guard<std::mutex> lk(m->mu);
    SpecKernel unused;
    mri_status st = spec_compile(m, 128, kStiffKind, 0, 0, &unused);
    if (st == MRI_OK && code_bytes) *code_bytes = m->last_code.size();
    return st;
}

mri_status mri_mech_code_hash(mri_mech *m, int method, int n_poly, int block_size,
                              uint64_t *hash)
{
    if (!hash) return fail(MRI_EINVAL, "hash is NULL");
    mri_status st = check_spec_request(m, method, n_poly, block_size);
    if (st != MRI_OK) return st;
    // compile and hash under one lock so that a concurrent compilation cannot
    // interleave
    std::lock_guard<std::mutex> lk(m->mu);
    SpecKernel unused;
    st = spec_compile(m, block_size, spec_kind(method), n_poly, 0, &unused);
    if (st != MRI_OK) return st;
    *hash = code_hash_bytes(m->last_code);
    return MRI_OK;
}

mri_status mri_mech_specialize(mri_mech *m, int block_size, int load, size_t *code_bytes)
{
    // the RK4 kernel with a constant forcing term (the explicit MIS/MRI-GARK case)
    return mri_mech_specialize_method(m, MRI_FAST_RK4, 1, block_size, load, code_bytes);
}

mri_status mri_table_create(const mri_table_desc *d, mri_table **out)
{
    if (!out) return fail(MRI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d || !d->c || !d->gamma) return fail(MRI_EINVAL, "table desc or its arrays are NULL");
    const int s = d->s, ng = d->n_gamma;
    if (s < 2 || s > 8) return fail(MRI_EINVAL, "s must be in [2, 8] (got %d)", s);
    if (ng < 1 || ng > 4) return fail(MRI_EINVAL, "n_gamma must be in [1, 4] (got %d)", ng);
    if (!finite_all(d->c, s) || !finite_all(d->gamma, ng * s * s))
        return fail(MRI_EINVAL, "non-finite table entry");
    if (d->c[0] != 0.0) return fail(MRI_EINVAL, "c_1 must be 0");
    for (int i = 1; i < s; ++i)
        if (!(d->c[i] > d->c[i - 1]))
            return fail(MRI_EINVAL, "explicit tables need strictly increasing c (stage %d)", i);
    for (int k = 0; k < ng; ++k)
        for (int i = 0; i < s; ++i)
            for (int j = i; j < s; ++j)
                if (d->gamma[((size_t)k * s + i) * s + j] != 0.0)
                    return fail(MRI_EINVAL, "gamma[%d][%d][%d] must be 0 (explicit table)", k, i, j);
    for (int i = 1; i < s; ++i) {
        double tot = 0.0;
        for (int k = 0; k < ng; ++k)
            for (int j = 0; j < i; ++j) tot += d->gamma[((size_t)k * s + i) * s + j] / (k + 1);
        const double dc = d->c[i] - d->c[i - 1];
        if (std::fabs(tot - dc) > 1e-12 * std::max(1.0, std::fabs(dc)))
            return fail(MRI_EINVAL, "row %d violates sum_j sum_k gamma/(k+1) = dc (%.3e vs %.3e)",
                        i, tot, dc);
    }
    std::unique_ptr<mri_table> t(new mri_table);
    t->s = s;
    t->ng = ng;
    t->c.assign(d->c, d->c + s);
    t->gamma.assign(d->gamma, d->gamma + (size_t)ng * s * s);
    *out = t.release();
    return MRI_OK;
}

void mri_table_destroy(mri_table *t) { delete t; }

mri_status mri_fast_stage(const mri_mech *mc, const mri_fast_opts *opts, int n_cells, int ld,
                          const double *y_in, double *y_out, int n_poly, const double *rho_poly,
                          double L, int32_t *status_out, int32_t *steps_out, mri_stream_t stream)
{
    mri_mech *m = const_cast<mri_mech *>(mc);
    if (!m) return fail(MRI_EINVAL, "mech is NULL");
    mri_status st = check_opts(m, opts);
    if (st != MRI_OK) return st;
    if (n_cells < 0 || ld < n_cells) return fail(MRI_EINVAL, "need 0 <= n_cells <= ld");
    if (ld > kMaxCells) return fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    if ((long long)ld * m->n > (1ll << 31) - 1)
        return fail(MRI_EINVAL, "n * ld exceeds 2^31 - 1 elements");
    if (n_poly < 0 || n_poly > 4) return fail(MRI_EINVAL, "n_poly must be in [0, 4]");
    if (n_poly > 0 && !rho_poly) return fail(MRI_EINVAL, "rho_poly is NULL with n_poly > 0");
    if (!(L > 0.0) || !std::isfinite(L)) return fail(MRI_EINVAL, "L must be positive and finite");
    if (n_cells == 0) return MRI_OK;
    if (!y_in || !y_out) return fail(MRI_EINVAL, "y_in or y_out is NULL");
    return fast_stage_impl(m, opts, n_cells, ld, y_in, y_out, n_poly, rho_poly, L, status_out,
                           steps_out, 0, (hipStream_t)stream);
}

mri_status mri_workspace_bytes(const mri_mech *m, const mri_table *t, int n_cells, int ld,
                               size_t *bytes)
{
    if (!m || !t || !bytes) return fail(MRI_EINVAL, "NULL argument");
    if (n_cells < 0 || ld < n_cells) return fail(MRI_EINVAL, "need 0 <= n_cells <= ld");
    if (ld > kMaxCells) return fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    *bytes = sizeof(double) * (size_t)m->n * (size_t)ld * (size_t)(t->s - 1 + t->ng);
    return MRI_OK;
}

mri_status mri_slow_step(const mri_mech *mc, const mri_table *t, const mri_fast_opts *opts,
                         mri_slow_rhs f_slow, void *user, double t0, double H, int n_cells,
                         int ld, double *y, void *ws, size_t ws_bytes, int32_t *status_out,
                         int32_t *steps_out, mri_stream_t stream)
{
    mri_mech *m = const_cast<mri_mech *>(mc);
    mri_status st = mri_internal_check_slow_step(m, t, opts, f_slow, t0, H, n_cells, ld);
    if (st != MRI_OK) return st;
    size_t need = 0;
    mri_workspace_bytes(m, t, n_cells, ld, &need);
    if (n_cells == 0) return MRI_OK;
    if (!y) return fail(MRI_EINVAL, "y is NULL");
    if (!ws || ws_bytes < need)
        return fail(MRI_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, need);
    const size_t vec = (size_t)m->n * ld;
    double *F = (double *)ws;                       // [s-1][n][ld]
    double *rho = F + (size_t)(t->s - 1) * vec;     // [ng][n][ld]
    return mri_internal_slow_step(m, t, opts, f_slow, user, t0, H, n_cells, ld, y, F, rho,
                                  status_out, steps_out, 1, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Adaptive slow steps (step doubling)
// ---------------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

mri_status mri_adaptive_workspace_bytes(const mri_mech *m, const mri_table *t, int n_cells,
                                        int ld, size_t *bytes)
{
    size_t base = 0;
    mri_status st = mri_workspace_bytes(m, t, n_cells, ld, &base);
    if (st != MRI_OK) return st;
    const size_t vec = sizeof(double) * (size_t)m->n * (size_t)ld;
    const size_t nb = (size_t)step_err_blocks(n_cells);
    *bytes = align256(base) + 2 * align256(vec) + 4 * align256(sizeof(int32_t) * (size_t)ld) +
             align256(nb * sizeof(double)) + align256(nb * sizeof(long long));
    return MRI_OK;
}

mri_status mri_adaptive_run(const mri_mech *mc, const mri_table *t, const mri_fast_opts *opts,
                            const mri_adapt_opts *a, mri_slow_rhs f_slow, void *user, double t0,
                            double t_end, int n_cells, int ld, double *y, void *ws,
                            size_t ws_bytes, int32_t *status_out, mri_adapt_stats *stats,
                            mri_stream_t stream)
{
    mri_mech *m = const_cast<mri_mech *>(mc);
    if (!m || !t) return fail(MRI_EINVAL, "mech or table is NULL");
    mri_status st = check_opts(m, opts);
    if (st != MRI_OK) return st;
    if (!a) return fail(MRI_EINVAL, "adaptive options are NULL");
    if (!f_slow) return fail(MRI_EINVAL, "slow RHS callback is NULL");
    const bool fin = std::isfinite(a->rtol) && std::isfinite(a->atol_Y) &&
                     std::isfinite(a->atol_T) && std::isfinite(a->H0) &&
                     std::isfinite(a->H_min) && std::isfinite(a->H_max);
    if (!fin || !(a->rtol >= 0.0) || !(a->atol_Y > 0.0) || !(a->atol_T > 0.0))
        return fail(MRI_EINVAL, "tolerances must be finite with atol > 0, rtol >= 0");
    if (!(a->H0 > 0.0) || !(a->H_min >= 0.0) || !(a->H_max >= 0.0) ||
        (a->H_max > 0.0 && a->H_max < a->H_min))
        return fail(MRI_EINVAL, "need H0 > 0, 0 <= H_min <= H_max (H_max = 0: unbounded)");
    if (a->order < 1 || a->order > 8) return fail(MRI_EINVAL, "order must be in [1, 8]");
    if (a->max_attempts < 1) return fail(MRI_EINVAL, "max_attempts must be >= 1");
    const double safety = a->safety == 0.0 ? 0.9 : a->safety;
    const double fac_min = a->fac_min == 0.0 ? 0.2 : a->fac_min;
    const double fac_max = a->fac_max == 0.0 ? 5.0 : a->fac_max;
    if (!(safety > 0.0 && safety <= 1.0) || !(fac_min > 0.0 && fac_min < 1.0) ||
        !(fac_max > 1.0 && std::isfinite(fac_max)))
        return fail(MRI_EINVAL, "need 0 < safety <= 1, 0 < fac_min < 1 < fac_max");
    if (!std::isfinite(t0) || !std::isfinite(t_end) || !(t_end > t0))
        return fail(MRI_EINVAL, "need finite t0 < t_end");
    if (n_cells < 0 || ld < n_cells) return fail(MRI_EINVAL, "need 0 <= n_cells <= ld");
    if (ld > kMaxCells) return fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    if ((long long)ld * m->n > (1ll << 31) - 1)
        return fail(MRI_EINVAL, "n * ld exceeds 2^31 - 1 elements");
    size_t need = 0, base = 0;
    mri_adaptive_workspace_bytes(m, t, n_cells, ld, &need);
    mri_workspace_bytes(m, t, n_cells, ld, &base);
    mri_adapt_stats loc{};
    mri_adapt_stats *sp = stats ? stats : &loc;
    *sp = mri_adapt_stats{};
    sp->t = t0;
    sp->H_next = a->H0;
    if (n_cells == 0) {
        sp->t = t_end;
        return MRI_OK;
    }
    if (!y) return fail(MRI_EINVAL, "y is NULL");
    if (!ws || ws_bytes < need)
        return fail(MRI_EINVAL, "workspace too small (%zu < %zu bytes)", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    // workspace: slow-step workspace | y_full | y_half | st_a st_b sp_a sp_b | partials
    const size_t vec = sizeof(double) * (size_t)m->n * (size_t)ld;
    const size_t ivec = align256(sizeof(int32_t) * (size_t)ld);
    const int nb = step_err_blocks(n_cells);
    char *p = (char *)ws;
    void *sws = p;
    p += align256(base);
    double *yf = (double *)p;
    p += align256(vec);
    double *yh = (double *)p;
    p += align256(vec);
    int32_t *st_a = (int32_t *)p, *st_b = (int32_t *)(p + ivec);
    int32_t *sp_a = (int32_t *)(p + 2 * ivec), *sp_b = (int32_t *)(p + 3 * ivec);
    p += 4 * ivec;
    double *part_w2 = (double *)p;
    p += align256(nb * sizeof(double));
    long long *part_steps = (long long *)p;
    if (status_out) HIP_TRY(hipMemsetAsync(status_out, 0, sizeof(int32_t) * n_cells, s));
    const int t_comp = m->kind == 0 ? m->n - 1 : -1;
    const double scale = 1.0 / (std::ldexp(1.0, a->order) - 1.0);
    const bool fixed = fixed_step(opts->method);
    std::vector<double> hw(nb);
    std::vector<long long> hs(nb);
    mri_fast_opts fo = *opts;
    // fixed-step fast methods keep the fast step size of the first step
    auto nsub_for = [&](double h) {
        return fixed ? std::max(1, (int)std::ceil(opts->n_sub * (h / a->H0) - 1e-9)) : opts->n_sub;
    };
    double tc = t0;
    double H = a->H_max > 0.0 ? std::min(a->H0, a->H_max) : a->H0;
    int attempts = 0;
    while (tc < t_end) {
        if (attempts >= a->max_attempts)
            return fail(MRI_EMAXSTEPS, "%d attempted steps did not reach t_end (t = %.17g)",
                        attempts, tc);
        ++attempts;
        double Hs = H;
        bool last = false;
        if (tc + Hs >= t_end - 1e-12 * (t_end - t0)) {
            Hs = t_end - tc;
            last = true;
        }
        HIP_TRY(hipMemcpyAsync(yf, y, vec, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(yh, y, vec, hipMemcpyDeviceToDevice, s));
        fo.n_sub = nsub_for(Hs);
        st = mri_slow_step(m, t, &fo, f_slow, user, tc, Hs, n_cells, ld, yf, sws, base, nullptr,
                           nullptr, stream);
        if (st != MRI_OK) return st;
        fo.n_sub = nsub_for(0.5 * Hs);
        st = mri_slow_step(m, t, &fo, f_slow, user, tc, 0.5 * Hs, n_cells, ld, yh, sws, base,
                           st_a, sp_a, stream);
        if (st != MRI_OK) return st;
        st = mri_slow_step(m, t, &fo, f_slow, user, tc + 0.5 * Hs, 0.5 * Hs, n_cells, ld, yh,
                           sws, base, st_b, sp_b, stream);
        if (st != MRI_OK) return st;
        HIP_TRY(launch_step_err(m->n, t_comp, n_cells, ld, yh, yf, scale, a->rtol, a->atol_Y,
                                a->atol_T, sp_a, sp_b, part_w2, part_steps, s));
        HIP_TRY(hipMemcpyAsync(hw.data(), part_w2, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hs.data(), part_steps, sizeof(long long) * nb,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double sum = 0.0;
        long long fast = 0;
        for (int b = 0; b < nb; ++b) {
            sum += hw[b];
            fast += hs[b];
        }
        double err = std::sqrt(sum / ((double)m->n * (double)n_cells));
        if (!std::isfinite(err)) err = HUGE_VAL;
        double fac = err == 0.0       ? fac_max
                     : err == HUGE_VAL ? fac_min
                                       : safety * std::pow(err, -1.0 / (a->order + 1));
        fac = std::min(fac_max, std::max(fac_min, fac));
        sp->err_last = err;
        if (err <= 1.0) {
            HIP_TRY(hipMemcpyAsync(y, yh, vec, hipMemcpyDeviceToDevice, s));
            if (status_out) HIP_TRY(launch_status_merge(n_cells, st_a, st_b, status_out, s));
            tc = last ? t_end : tc + Hs;
            ++sp->accepted;
            sp->H_last = Hs;
            sp->fast_steps += fast;
        } else {
            ++sp->rejected;
        }
        H = Hs * fac;
        if (a->H_max > 0.0) H = std::min(H, a->H_max);
        sp->t = tc;
        sp->H_next = H;
        if (err > 1.0 && H < a->H_min)
            return fail(MRI_EMAXSTEPS, "step size %.3g fell below H_min at t = %.17g", H, tc);
    }
    return MRI_OK;
}

mri_status mri_forcing_assemble(const mri_table *t, int stage, int n, int ld, const double *F,
                                double *rho, mri_stream_t stream)
{
    if (!t || !F || !rho) return fail(MRI_EINVAL, "NULL argument");
    if (stage < 1 || stage >= t->s) return fail(MRI_EINVAL, "stage must be in [1, s)");
    if (n < 1 || ld < 0) return fail(MRI_EINVAL, "bad n / ld");
    if (ld == 0) return MRI_OK;
    const double dc = t->c[stage] - t->c[stage - 1];
    ForcingCoef coef{};
    for (int k = 0; k < t->ng; ++k)
        for (int j = 0; j < stage; ++j)
            coef.c[k * 8 + j] = t->gamma[((size_t)k * t->s + stage) * t->s + j] / dc;
    const long long vec = (long long)n * ld;
    HIP_TRY(launch_forcing(vec, t->ng, stage, F, vec, coef, rho, (hipStream_t)stream));
    return MRI_OK;
}

int mri_advdiff_slow_rhs(double t, const double *y, double *fy, int n_cells, int ld, void *user,
                         mri_stream_t stream)
{
    (void)t;
    const mri_advdiff_params *p = (const mri_advdiff_params *)user;
    if (!p || !y || !fy) return -1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->n_comp < 1) return -2;
    if ((long long)p->nx * p->ny * p->nz != n_cells || ld < n_cells) return -3;
    if (!(p->dx > 0.0)) return -4;
    if (p->ny > 65535 || p->nz > 65535) return -6;
    if (launch_advdiff(p->nx, p->ny, p->nz, p->n_comp, ld, p->u, p->D, p->dx, y, fy,
                       (hipStream_t)stream) != hipSuccess)
        return -5;
    return 0;
}

int mri_linear_slow_rhs(double t, const double *y, double *fy, int n_cells, int ld, void *user,
                        mri_stream_t stream)
{
    (void)t;
    const mri_mech *m = (const mri_mech *)user;
    if (!m || m->kind != 1 || !y || !fy) return -1;
    if (ensure_device(const_cast<mri_mech *>(m)) != MRI_OK) return -6;
    if (launch_lin_apply(m->n, m->d_A, n_cells, ld, y, fy, (hipStream_t)stream) != hipSuccess)
        return -5;
    return 0;
}

mri_status mri_selftest_exp2(const double *x, double *y, int n, mri_stream_t stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) return fail(MRI_EINVAL, "bad arguments");
    if (n == 0) return MRI_OK;
    HIP_TRY(launch_exp2(x, y, n, (hipStream_t)stream));
    return MRI_OK;
}

mri_status mri_selftest_exp2_t256(const double *x, double *y, int n, mri_stream_t stream)
{
    if (n < 0 || (n > 0 && (!x || !y))) return fail(MRI_EINVAL, "bad arguments");
    if (n == 0) return MRI_OK;
    HIP_TRY(launch_exp2_t256(x, y, n, (hipStream_t)stream));
    return MRI_OK;
}

mri_status mri_stiffness_check(const mri_mech *mc, int n_cells, int ld, const double *y, double h,
                               double limit, double *bound_out, int32_t *status,
                               mri_stream_t stream)
{
    mri_mech *m = const_cast<mri_mech *>(mc);
    if (!m) return fail(MRI_EINVAL, "mech is NULL");
    if (m->kind != 0) return fail(MRI_EUNSUPPORTED, "the monitor needs a chemistry mechanism");
    if (n_cells < 0 || ld < n_cells) return fail(MRI_EINVAL, "need 0 <= n_cells <= ld");
    if (ld > kMaxCells) return fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    if ((long long)ld * m->n > (1ll << 31) - 1)
        return fail(MRI_EINVAL, "n * ld exceeds 2^31 - 1 elements");
    if (!(h >= 0.0) || !std::isfinite(h) || !(limit >= 0.0) || std::isnan(limit))
        return fail(MRI_EINVAL, "need finite h >= 0 and limit >= 0");
    if (n_cells == 0) return MRI_OK;
    if (!y) return fail(MRI_EINVAL, "y is NULL");
    mri_status st = ensure_device(m);
    if (st != MRI_OK) return st;
    HIP_TRY(launch_gen_stiff(m->gm, n_cells, ld, y, h, limit, bound_out, status, nullptr, 1,
                             MRI_CELL_STIFF, (hipStream_t)stream));
    return MRI_OK;
}

mri_status mri_status_count(const int32_t *status, int n_cells, int32_t mask, int64_t *n_bad,
                            mri_stream_t stream)
{
    if (!n_bad) return fail(MRI_EINVAL, "n_bad is NULL");
    if (n_cells < 0 || n_cells > kMaxCells)
        return fail(MRI_EINVAL, "need 0 <= n_cells <= 2^31 - 1024");
    *n_bad = 0;
    if (n_cells == 0) return MRI_OK;
    if (!status) return fail(MRI_EINVAL, "status is NULL");
    hipStream_t s = (hipStream_t)stream;
    // one device counter per GPU, allocated on the first call there and kept
    // until the process ends; the lock spans the whole (synchronizing) call, so
    // concurrent calls take turns instead of sharing the counter
    static std::mutex mu;
    static unsigned long long *counter[64] = {};
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(MRI_EUNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lk(mu);
    if (!counter[dev]) HIP_TRY(hipMalloc(&counter[dev], sizeof(unsigned long long)));
    unsigned long long *d = counter[dev];
    unsigned long long h = 0;
    hipError_t e = launch_fill_u64(d, 1, 0ull, s);
    if (e == hipSuccess) e = launch_status_count(status, n_cells, mask, d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(MRI_EHIP, "status count failed: %s", hipGetErrorString(e));
    *n_bad = (int64_t)h;
    return MRI_OK;
}

// ---------------------------------------------------------------------------
// Batched uneven sets: persistent work-queue kernel (specialized kernels).
// ---------------------------------------------------------------------------
mri_status mri_batch_plan_create(const mri_mech *mc, const mri_fast_opts *opts, int n_sets,
                                 const int64_t *set_offsets, mri_batch_plan **out)
{
    mri_mech *m = const_cast<mri_mech *>(mc);
    if (!out) return fail(MRI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!m) return fail(MRI_EINVAL, "mech is NULL");
    mri_status st = check_opts(m, opts);
    if (st != MRI_OK) return st;
    if (opts->method != MRI_FAST_ZONNEVELD43)
        return fail(MRI_EINVAL, "batched plans integrate with the adaptive Zonneveld method");
    if (m->kind != 0) return fail(MRI_EUNSUPPORTED, "batched plans need a chemistry mechanism");
    if (n_sets < 1 || !set_offsets) return fail(MRI_EINVAL, "need n_sets >= 1 and set_offsets");
    if (set_offsets[0] != 0) return fail(MRI_EINVAL, "set_offsets[0] must be 0");
    for (int i = 0; i < n_sets; ++i)
        if (set_offsets[i + 1] < set_offsets[i])
            return fail(MRI_EINVAL, "set_offsets must be non-decreasing (set %d)", i);
    std::unique_ptr<mri_batch_plan> p(new mri_batch_plan);
    p->mech = m;
    p->opts = *opts;
    p->n_sets = n_sets;
    p->off.assign(set_offsets, set_offsets + n_sets + 1);
    p->n_total = p->off.back();
    HIP_TRY(hipMalloc(&p->d_off, sizeof(long long) * (n_sets + 1)));
    HIP_TRY(hipMemcpy(p->d_off, p->off.data(), sizeof(long long) * (n_sets + 1),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&p->d_L, sizeof(double) * n_sets));
    HIP_TRY(hipMalloc(&p->d_counters, sizeof(unsigned long long) * 3));
    *out = p.release();
    return MRI_OK;
}

void mri_batch_plan_destroy(mri_batch_plan *p) { delete p; }

mri_status mri_batch_plan_tile(const mri_batch_plan *p, int *block_size, int *n_blocks)
{
    if (!p || !block_size || !n_blocks) return fail(MRI_EINVAL, "NULL argument");
    if (!p->tuned) return fail(MRI_EINVAL, "plan has not run yet");
    *block_size = p->wg;
    *n_blocks = p->n_blocks;
    return MRI_OK;
}

}  // extern "C"

// Enqueue one persistent launch (counter reset by a fill kernel, then the
// work-queue kernel) over the first n_total cells on stream s.
static mri_status batch_enqueue(mri_batch_plan *p, int wg, int n_blocks, const SpecVariant &var,
                                long long n_total, const double *yin, double *yout,
                                long long ld, int n_poly, const double *rho, int32_t *status,
                                int32_t *steps, int32_t *rejects, hipStream_t s)
{
    hipFunction_t fn = nullptr;
    mri_status st = spec_get(p->mech, wg, 2, n_poly, &fn, var);
    if (st != MRI_OK) return st;
    HIP_TRY(launch_fill_u64(p->d_counters, 3, 0ull, s));
    BatchArgs a;
    a.yin = yin;
    a.yout = yout;
    a.rho = rho;
    a.set_off = p->d_off;
    a.set_L = p->d_L;
    a.status = status;
    a.steps = steps;
    a.rejects = rejects;
    a.counter = p->d_counters;
    a.lane_steps = p->d_counters + 1;
    a.issued_steps = p->d_counters + 2;
    a.n_total = n_total;
    a.ld = ld;
    a.n_sets = p->n_sets;
    a.o = ZvOpts{p->opts.rtol, p->opts.atol_Y, p->opts.atol_T, p->opts.max_steps};
    void *args[] = {&a};
    HIP_TRY(hipModuleLaunchKernel(fn, (unsigned)n_blocks, 1, 1, wg, 1, 1, 0, s, args, nullptr));
    return MRI_OK;
}

static int n_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    return cus > 0 ? cus : 256;
}

// FNV-1a over a byte string (the mechanism's literal block identifies it).
static uint64_t fnv1a(const std::string &b)
{
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : b) h = (h ^ c) * 1099511628211ull;
    return h;
}

// Tuning results by (mechanism, S, R, fast method, forcing terms, tolerances,
// size class = floor(log2(cells)), device architecture), in memory and in a
// text file: MRI_TUNE_CACHE names it
// ("off" disables it), else $XDG_CACHE_HOME/libmri/batch_tune.txt or
// $HOME/.cache/libmri/batch_tune.txt.  A line holds the key and the choice:
// threads per block, grid factor, waves per SIMD, exponential, window, ms.
struct TuneChoice {
    int wg = 0, factor = 1;
    SpecVariant var;
    float ms = 0.0f;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneChoice> g_tune;
static bool g_tune_loaded = false;

static std::string tune_cache_path()
{
    if (const char *e = std::getenv("MRI_TUNE_CACHE")) return std::string(e) == "off" ? "" : e;
    if (const char *x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/libmri/batch_tune.txt";
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/libmri/batch_tune.txt";
    return "";
}

static std::string tune_key(const mri_batch_plan *p, int n_poly)
{
    char b[256];
    mri_mech *m = p->mech;
    uint64_t defs_hash = 0;
    {
        // the literal block is generated on the first compilation; generate it
        // here when no kernel has been compiled yet, so that the key is the same
        // before and after
        std::lock_guard<std::mutex> lk(m->mu);
        if (m->defs.empty()) m->defs = make_defs(*m);
        defs_hash = fnv1a(m->defs);
    }
    int size_class = 0;
    while (size_class < 62 && (2ll << size_class) <= p->n_total) ++size_class;
    snprintf(b, sizeof b, "mech=%016llx S=%d R=%d method=%d np=%d rtol=%a atolY=%a atolT=%a "
             "max_steps=%d log2cells=%d arch=%s",
             (unsigned long long)defs_hash, m->S, m->R, p->opts.method, n_poly,
             p->opts.rtol, p->opts.atol_Y, p->opts.atol_T, p->opts.max_steps, size_class,
             device_arch().c_str());
    return b;
}

// Looks a choice up (loading the file on first use); caller holds g_tune_mu.
static bool tune_lookup(const std::string &key, TuneChoice *c)
{
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        const std::string path = tune_cache_path();
        if (!path.empty()) {
            std::ifstream in(path);
            for (std::string line; std::getline(in, line);) {
                const size_t tab = line.find('\t');
                if (tab == std::string::npos) continue;
                TuneChoice t;
                if (sscanf(line.c_str() + tab + 1, "%d %d %d %d %d %f", &t.wg, &t.factor,
                           &t.var.wpe, &t.var.exp_table, &t.var.group, &t.ms) == 6 &&
                    (t.wg == 64 || t.wg == 128 || t.wg == 256) && t.factor >= 1 &&
                    t.factor <= 4)
                    g_tune[line.substr(0, tab)] = t;
            }
        }
    }
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *c = it->second;
    return true;
}

static void tune_store(const std::string &key, const TuneChoice &c)
{
    g_tune[key] = c;
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        // create the directory chain (best effort; an unwritable cache is skipped)
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    std::ofstream out(path, std::ios::app);
    if (out)
        out << key << '\t' << c.wg << ' ' << c.factor << ' ' << c.var.wpe << ' '
            << c.var.exp_table << ' ' << c.var.group << ' ' << c.ms << '\n';
}

static mri_status resident_blocks(mri_batch_plan *p, int wg, int n_poly, const SpecVariant &var,
                                  int *nb)
{
    hipFunction_t fn = nullptr;
    mri_status st = spec_get(p->mech, wg, 2, n_poly, &fn, var);
    if (st != MRI_OK) return st;
    int b = 0;
    HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, wg, 0));
    *nb = std::max(1, b) * n_cus();
    return MRI_OK;
}

// Autotuner of the persistent work-queue launch, timed on a prefix of the sets
// holding about 1/8 of the cells (at least 64k when available):
//   1. tile: 64 / 128 / 256 threads per block x grid = 1x or 2x the resident
//      capacity the occupancy query reports, with the built-in tiling;
//   2. register / LDS tiling at the best block size: the other number of waves
//      per SIMD (which moves the exponential between its LDS table and the
//      polynomial), the other exponential alone, and scheduling windows of 1
//      and 4 rate evaluations, each at both grid factors.
// The fastest choice is kept and cached (see tune_key); a plan created later
// with the same key takes it without timing anything.
static mri_status batch_tune(mri_batch_plan *p, const double *yin, double *yout, long long ld,
                             int n_poly, const double *rho, hipStream_t s)
{
    if (p->opts.block_size) {
        p->wg = p->opts.block_size;
        p->var = SpecVariant();
        mri_status st = resident_blocks(p, p->wg, n_poly, p->var, &p->n_blocks);
        if (st != MRI_OK) return st;
        p->tuned = true;
        return MRI_OK;
    }
    const std::string key = tune_key(p, n_poly);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        TuneChoice c;
        if (tune_lookup(key, &c)) {
            int nb = 0;
            mri_status st = resident_blocks(p, c.wg, n_poly, c.var, &nb);
            if (st == MRI_OK) {
                p->wg = c.wg;
                p->var = c.var;
                p->n_blocks = nb * c.factor;
                p->tune_ms = c.ms;
                p->tuned = p->from_cache = true;
                p->tune_log.clear();
                return MRI_OK;
            }
        }
    }
    long long target = std::max<long long>(std::min<long long>(p->n_total, 65536), p->n_total / 8);
    int k = 1;
    while (k < p->n_sets && p->off[k] < target) ++k;
    const long long n_sample = p->off[k];
    struct Events {   // destroyed on every return path
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events()
        {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    HIP_TRY(hipEventCreate(&ev.e0));
    HIP_TRY(hipEventCreate(&ev.e1));
    float best = 1e30f;
    TuneChoice pick;
    p->tune_log.clear();
    auto trial = [&](int wg, const SpecVariant &var) -> mri_status {
        int nb = 0;
        mri_status st = resident_blocks(p, wg, n_poly, var, &nb);
        if (st != MRI_OK) return st;
        for (int f : {1, 2}) {
            HIP_TRY(hipEventRecord(ev.e0, s));
            st = batch_enqueue(p, wg, nb * f, var, n_sample, yin, yout, ld, n_poly, rho, nullptr,
                               nullptr, nullptr, s);
            if (st != MRI_OK) return st;
            HIP_TRY(hipEventRecord(ev.e1, s));
            HIP_TRY(hipEventSynchronize(ev.e1));
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, ev.e0, ev.e1));
            p->tune_log.push_back({wg, nb * f, var, ms});
            if (ms < best) {
                best = ms;
                pick.wg = wg;
                pick.factor = f;
                pick.var = var;
                pick.ms = ms;
            }
        }
        return MRI_OK;
    };
    for (int wg : {64, 128, 256}) {
        mri_status st = trial(wg, SpecVariant());
        if (st != MRI_OK) return st;
    }
    // register / LDS tiling variants at the best block size; a variant the
    // compiler rejects (e.g. registers that do not fit) is skipped
    SpecVariant v1, v2, v3, v4;
    v1.wpe = (p->mech->S < 40) ? 1 : 2;
    v2.exp_table = 0;
    v3.group = 1;
    v4.group = 4;
    const int wg_best = pick.wg;
    for (const SpecVariant &v : {v1, v2, v3, v4}) {
        mri_status st = trial(wg_best, v);
        if (st == MRI_ECOMPILE) continue;
        if (st != MRI_OK) return st;
    }
    int nb = 0;
    mri_status st = resident_blocks(p, pick.wg, n_poly, pick.var, &nb);
    if (st != MRI_OK) return st;
    p->wg = pick.wg;
    p->var = pick.var;
    p->n_blocks = nb * pick.factor;
    p->tune_ms = pick.ms;
    p->tuned = true;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_store(key, pick);
    return MRI_OK;
}

extern "C" mri_status mri_batch_run(mri_batch_plan *p, const double *y_in, double *y_out,
                                    int64_t ld, int n_poly, const double *rho_poly,
                                    const double *L_per_set, int32_t *status_out,
                                    int32_t *steps_out, int32_t *rejects_out,
                                    mri_stream_t stream)
{
    if (!p) return fail(MRI_EINVAL, "plan is NULL");
    if (ld < p->n_total) return fail(MRI_EINVAL, "ld < total cells");
    if (ld > kMaxCells) return fail(MRI_EINVAL, "ld exceeds 2^31 - 1024 cells");
    if (ld * (int64_t)p->mech->n > (1ll << 31) - 1)
        return fail(MRI_EINVAL, "n * ld exceeds 2^31 - 1 elements");
    if (n_poly < 0 || n_poly > 4 || (n_poly > 0 && !rho_poly))
        return fail(MRI_EINVAL, "bad n_poly / rho_poly");
    if (!L_per_set) return fail(MRI_EINVAL, "L_per_set is NULL");
    for (int i = 0; i < p->n_sets; ++i)
        if (!(L_per_set[i] > 0.0) || !std::isfinite(L_per_set[i]))
            return fail(MRI_EINVAL, "L_per_set[%d] must be positive and finite", i);
    if (p->n_total == 0) return MRI_OK;
    if (!y_in || !y_out) return fail(MRI_EINVAL, "y_in or y_out is NULL");
    if (y_in == y_out) return fail(MRI_EINVAL, "batched runs need y_out distinct from y_in");
    mri_status st = ensure_device(p->mech);
    if (st != MRI_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(p->d_L, L_per_set, sizeof(double) * p->n_sets, hipMemcpyHostToDevice, s));
    if (!p->tuned) {
        st = batch_tune(p, y_in, y_out, ld, n_poly, rho_poly, s);
        if (st != MRI_OK) return st;
    }
    const std::vector<uintptr_t> key = {(uintptr_t)y_in, (uintptr_t)y_out, (uintptr_t)ld,
                                        (uintptr_t)spec_key(p->wg, 2, n_poly, p->var),
                                        (uintptr_t)n_poly, (uintptr_t)rho_poly,
                                        (uintptr_t)status_out, (uintptr_t)steps_out,
                                        (uintptr_t)rejects_out, (uintptr_t)p->wg,
                                        (uintptr_t)p->n_blocks};
    if (!p->exec || key != p->graph_key) {
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
        // compile outside the capture
        hipFunction_t fn = nullptr;
        st = spec_get(p->mech, p->wg, 2, n_poly, &fn, p->var);
        if (st != MRI_OK) return st;
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        st = batch_enqueue(p, p->wg, p->n_blocks, p->var, p->n_total, y_in, y_out, ld, n_poly,
                           rho_poly, status_out, steps_out, rejects_out, p->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
        if (st != MRI_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (ce != hipSuccess) return fail(MRI_EHIP, "capture failed: %s", hipGetErrorString(ce));
        p->graph = g;
        HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
        p->graph_key = key;
    }
    HIP_TRY(hipGraphLaunch(p->exec, s));
    ++c_fast;
    c_cells += p->n_total;
    return MRI_OK;
}

extern "C" mri_status mri_batch_plan_tune_log(const mri_batch_plan *p, int max_entries,
                                              mri_tune_trial *trials, int *n_entries,
                                              int *from_cache, mri_tune_trial *choice)
{
    if (!p || !n_entries) return fail(MRI_EINVAL, "NULL argument");
    if (max_entries < 0 || (max_entries > 0 && !trials))
        return fail(MRI_EINVAL, "bad trial buffer");
    *n_entries = (int)p->tune_log.size();
    for (int i = 0; i < std::min(max_entries, *n_entries); ++i) {
        const auto &t = p->tune_log[i];
        trials[i] = mri_tune_trial{t.wg, t.blocks, t.var.wpe, t.var.exp_table, t.var.group, t.ms};
    }
    if (from_cache) *from_cache = p->from_cache ? 1 : 0;
    if (choice)
        *choice = mri_tune_trial{p->wg, p->n_blocks, p->var.wpe, p->var.exp_table, p->var.group,
                                 p->tune_ms};
    return MRI_OK;
}

extern "C" mri_status mri_batch_plan_code_hash(const mri_batch_plan *p, int n_poly,
                                               uint64_t *hash)
{
    if (!p || !hash) return fail(MRI_EINVAL, "NULL argument");
    if (n_poly < 0 || n_poly > 4) return fail(MRI_EINVAL, "n_poly must be in [0, 4]");
    const int wg = p->wg ? p->wg : (p->opts.block_size ? p->opts.block_size : 128);
    std::lock_guard<std::mutex> lk(p->mech->mu);
    SpecKernel unused;
    mri_status st = spec_compile(p->mech, wg, 2, n_poly, 0, &unused, p->var);
    if (st != MRI_OK) return st;
    *hash = code_hash_bytes(p->mech->last_code);
    return MRI_OK;
}

extern "C" mri_status mri_batch_lane_stats(const mri_batch_plan *p, uint64_t *useful,
                                           uint64_t *issued, mri_stream_t stream)
{
    if (!p || !useful || !issued) return fail(MRI_EINVAL, "NULL argument");
    unsigned long long h[3] = {0, 0, 0};
    HIP_TRY(hipMemcpyAsync(h, p->d_counters, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    *useful = h[1];
    *issued = h[2];
    return MRI_OK;
}
