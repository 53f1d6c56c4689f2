// Run-time specialization of the streaming kernel for one pass program.
//
// The paper generates the source of one kernel per merged plan and compiles it at run time
// (Section 5).  Here the generated source is the precompiled kernel's own code with the
// program written in as constants: every operation is the shared operation switch
// (sg_stream_ops.inc) behind a constant `op`, so the compiler removes the dispatch, indexes
// registers statically and keeps only the registers the program uses.  hiprtc compiles it
// for the device; kernels are cached per device and program (operations, constants, unroll
// and block bound), so a program pays the compilation once per process.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sg_runtime.h"
#include "sg_rtc_headers.h"  // generated at build time: the kernel headers as strings

using namespace sg;

namespace sgrt {

namespace {

struct JitKernel {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    std::map<std::pair<int, size_t>, int> occ;  // (block, LDS bytes) -> blocks per CU
};

std::mutex g_mu;
std::map<std::tuple<int, std::string>, JitKernel*> g_cache;  // (device, source) -> kernel

// A predicate followed by the check that pops it (outside the compacted space, whose checks
// are resolved after the scan) becomes one CHK_PRED operation.
std::vector<SgOp> fuse_checks(const InstPlan& ip) {
    std::vector<SgOp> out;
    for (size_t i = 0; i < ip.prog.size(); ++i) {
        const SgOp& p = ip.prog[i];
        const bool is_pred = p.code == P_FINITE || p.code == P_CMP_F || p.code == P_CMP_I || p.code == P_RANGE_F ||
                             p.code == P_RANGE_I;
        if (is_pred && i + 1 < ip.prog.size()) {
            const SgOp& c = ip.prog[i + 1];
            if ((c.code == CHK_ALL || c.code == CHK_ANY) && (c.sp == 0 || c.sp != ip.scan_space)) {
                SgOp f{};
                f.code = CHK_PRED;
                f.pad = p.code;
                f.sp2 = p.code == P_CMP_F || p.code == P_CMP_I ? p.aux : 0;
                f.a = p.a;
                f.c0 = p.c0;
                f.c1 = p.c1;
                f.dst = c.code == CHK_ALL ? 0 : 1;
                f.sp = c.sp;
                f.aux = c.aux;
                out.push_back(f);
                ++i;
                continue;
            }
        }
        out.push_back(p);
    }
    return out;
}

std::string program_source(const InstPlan& ip) {
    std::string s = "// generated: one pass program, operations as constants\n";
    char buf[320];
    for (const SgOp& o : fuse_checks(ip)) {
        uint32_t c0, c1;
        std::memcpy(&c0, &o.c0, 4);
        std::memcpy(&c1, &o.c1, 4);
        std::snprintf(buf, sizeof(buf),
                      "{\n  SgOp op;\n  op.code = %u; op.dst = %u; op.a = %u; op.b = %u; op.sp = %u; op.sp2 = %u; "
                      "op.aux = %u; op.pad = %u;\n  op.c0.i = (int32_t)0x%08xu; op.c1.i = (int32_t)0x%08xu;\n"
                      "  const uint8_t code = %u;\n",
                      o.code, o.dst, o.a, o.b, o.sp, o.sp2, o.aux, o.pad, c0, c1, o.code);
        s += buf;
        s += "#include \"sg_stream_ops.inc\"\n}\n";
    }
    return s;
}

std::string unit_source(const InstPlan& ip, int unroll, int lb) {
    // sources a sortedness check reads past the end of a wave's part (their next element is
    // prefetched with the sub-tile; no other source needs it)
    int nbr = 0;
    for (const SgOp& o : ip.prog)
        if (o.code == CHK_SORTED_F || o.code == CHK_SORTED_I) nbr |= 1 << (o.b & 7);
    char buf[640];
    std::snprintf(buf, sizeof(buf),
                  "#define SG_PROGRAM_INC \"sg_program_gen.inc\"\n#define SG_GEN_HAS_SCAN %d\n#define SG_GEN_NIN %d\n"
                  "#define SG_GEN_NSLOTS %d\n#define SG_GEN_NSUMS %d\n#define SG_GEN_NBR_MASK 0x%x\n"
                  "#include \"sg_stream_kernel.h\"\n"
                  "// instantiated through the name expression sg::stream_kernel<%d, true, %d, 1>\n",
                  ip.scan_space != 0 ? 1 : 0, (int)ip.sources.size(), (int)ip.slot_kind.size(), ip.nsum, nbr, unroll, lb);
    return buf;
}

}  // namespace

sg_status jit_kernel(sg_ctx_s* ctx, const InstPlan& ip, int unroll, int block, void** handle) {
    const int lb = block <= 256 ? 256 : block <= 512 ? 512 : 1024;  // register budget follows the block
    const std::string prog = program_source(ip);
    const std::string unit = unit_source(ip, unroll, lb);
    const auto key = std::make_tuple(ctx->device, unit + prog);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        *handle = it->second;
        return SG_OK;
    }
    // SG_JIT_DUMP=<directory>: write each generated unit and program there (for inspection
    // with an offline compiler)
    if (const char* dump = std::getenv("SG_JIT_DUMP")) {
        char path[512];
        const size_t id = std::hash<std::string>{}(unit + prog);
        std::snprintf(path, sizeof(path), "%s/sg_unit_%016zx.hip", dump, id);
        if (FILE* f = std::fopen(path, "w")) { std::fputs(unit.c_str(), f); std::fclose(f); }
        std::snprintf(path, sizeof(path), "%s/sg_program_%016zx.inc", dump, id);
        if (FILE* f = std::fopen(path, "w")) { std::fputs(prog.c_str(), f); std::fclose(f); }
    }
    std::vector<const char*> hdr_src, hdr_name;
    for (int i = 0; i < SG_RTC_NHEADERS; ++i) {
        hdr_src.push_back(SG_RTC_HEADER_TEXT[i]);
        hdr_name.push_back(SG_RTC_HEADER_NAME[i]);
    }
    hdr_src.push_back(prog.c_str());
    hdr_name.push_back("sg_program_gen.inc");
    hiprtcProgram rp;
    if (hiprtcCreateProgram(&rp, unit.c_str(), "sg_specialized.hip", (int)hdr_src.size(), hdr_src.data(),
                            hdr_name.data()) != HIPRTC_SUCCESS)
        return fail(ctx, SG_E_DEVICE, "hiprtc: create program");
    char expr[96];
    std::snprintf(expr, sizeof(expr), "&sg::stream_kernel<%d, true, %d, 1>", unroll, lb);
    (void)hiprtcAddNameExpression(rp, expr);
    char arch[64];
    std::snprintf(arch, sizeof(arch), "--offload-arch=%s", ctx->arch.c_str());
    const char* opts[] = {arch, "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult cr = hiprtcCompileProgram(rp, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (cr != HIPRTC_SUCCESS) {
        size_t n = 0;
        (void)hiprtcGetProgramLogSize(rp, &n);
        std::string log(n, '\0');
        if (n) (void)hiprtcGetProgramLog(rp, &log[0]);
        (void)hiprtcDestroyProgram(&rp);
        return fail(ctx, SG_E_DEVICE, ("hiprtc: compile failed: " + log.substr(0, 600)).c_str());
    }
    const char* lowered = nullptr;
    std::string name;
    if (hiprtcGetLoweredName(rp, expr, &lowered) == HIPRTC_SUCCESS && lowered) name = lowered;
    size_t csize = 0;
    (void)hiprtcGetCodeSize(rp, &csize);
    std::vector<char> code(csize);
    if (csize) (void)hiprtcGetCode(rp, code.data());
    (void)hiprtcDestroyProgram(&rp);
    if (name.empty() || csize == 0) return fail(ctx, SG_E_DEVICE, "hiprtc: no code or kernel name");
    auto* k = new JitKernel();
    if (hipModuleLoadData(&k->mod, code.data()) != hipSuccess ||
        hipModuleGetFunction(&k->fn, k->mod, name.c_str()) != hipSuccess) {
        if (k->mod) (void)hipModuleUnload(k->mod);
        delete k;
        return fail(ctx, SG_E_DEVICE, "specialized kernel: module load failed");
    }
    g_cache[key] = k;
    *handle = k;
    return SG_OK;
}

int jit_occupancy(void* handle, int block, size_t lds) {
    auto* k = (JitKernel*)handle;
    std::lock_guard<std::mutex> lock(g_mu);
    auto key = std::make_pair(block, lds);
    auto it = k->occ.find(key);
    if (it != k->occ.end()) return it->second;
    int nb = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k->fn, block, lds) != hipSuccess || nb < 1) nb = 1;
    k->occ[key] = nb;
    return nb;
}

hipError_t jit_launch(void* handle, const StreamArgs& a, int grid, int block, size_t lds, hipStream_t s,
                      hipEvent_t e0, hipEvent_t e1) {
    auto* k = (JitKernel*)handle;
    size_t size = sizeof(StreamArgs);
    void* extra[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, (void*)&a, HIP_LAUNCH_PARAM_BUFFER_SIZE, &size,
                     HIP_LAUNCH_PARAM_END};
    if (e0)  // work sizes in threads
        return hipExtModuleLaunchKernel(k->fn, (uint32_t)grid * (uint32_t)block, 1, 1, (uint32_t)block, 1, 1, lds, s,
                                        nullptr, extra, e0, e1, 0);
    return hipModuleLaunchKernel(k->fn, (unsigned)grid, 1, 1, (unsigned)block, 1, 1, (unsigned)lds, s, nullptr, extra);
}

}  // namespace sgrt
