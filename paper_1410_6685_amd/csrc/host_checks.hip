// Host evaluation of device arithmetic and of the planner's register programs, exported for
// CPU tests.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/safegpu.h"
#include "sg_exp.h"
#include "sg_runtime.h"

extern "C" sg_status sg_host_exp_rn(const float* t, float* out, int64_t n, int64_t* slow) {
    if ((!t || !out) && n > 0) return SG_E_INVALID;
    int s = 0;
    for (int64_t i = 0; i < n; ++i) out[i] = sgx::exp_rn(t[i], &s);
    if (slow) *slow = s;
    return SG_OK;
}

// Compile an expression agent into the register program a map gives it (x in register 0, the
// result back in register 0, registers 1 .. registers-1 free) and run that program on the host
// with binary32 operations, element by element.  *nops receives the program length.
// SG_E_UNSUPPORTED when the expression needs more registers than given.
extern "C" sg_status sg_host_expr_run(const char* text, int32_t registers, const float* x, float* out, int64_t n,
                                      int32_t* nops) {
    using namespace sg;
    if (!text || registers < 1 || registers > 64 || ((!x || !out) && n > 0)) return SG_E_INVALID;
    std::vector<sgrt::ExprNode> e;
    int root = -1;
    std::string why;
    if (!sgrt::parse_expr(text, e, &root, &why)) return SG_E_INVALID;
    std::vector<int> temps;
    for (int r = 1; r < registers; ++r) temps.push_back(r);
    if ((int)temps.size() > sgrt::expr_temps(e, root)) temps.resize(sgrt::expr_temps(e, root));
    std::vector<SgOp> prog;
    if (!sgrt::emit_expr(prog, e, root, 0, temps)) return SG_E_UNSUPPORTED;
    if (nops) *nops = (int32_t)prog.size();
    std::vector<float> R(registers);
    for (int64_t i = 0; i < n; ++i) {
        for (auto& v : R) v = std::nanf("");  // nothing but x is defined on entry
        R[0] = x[i];
        for (const SgOp& o : prog) {
            float& a = R[o.a];
            const float c = o.c0.f;
            switch (o.code) {
                case MOV: R[o.dst] = R[o.a]; break;
                case F_CONST: a = c; break;
                case F_ADDC: a = a + c; break;
                case F_MULC: a = a * c; break;
                case F_DIVC: a = a / c; break;
                case F_RDIVC: a = c / a; break;
                case F_NEG: a = -a; break;
                case F_ABS: a = std::fabs(a); break;
                case F_SQRT: a = std::sqrt(a); break;
                case F_EXP: a = sgx::exp_rn(a); break;
                case F_ADD: a = a + R[o.b]; break;
                case F_SUB: a = a - R[o.b]; break;
                case F_MUL: a = a * R[o.b]; break;
                case F_DIV: a = a / R[o.b]; break;
                default: return SG_E_INVALID;
            }
        }
        out[i] = R[0];
    }
    return SG_OK;
}
