// User element functions written as arithmetic expressions in x (agents of type FUNCTION,
// Section 3.2; the paper compiles such agents into the kernel it generates, Section 5).
//
// Grammar (whitespace ignored):
//     expr    := term (("+" | "-") term)*
//     term    := unary (("*" | "/") unary)*
//     unary   := "-" unary | primary
//     primary := number | "x" | "(" expr ")" | ("sqrt" | "abs" | "exp") "(" expr ")"
// Every literal is rounded to binary32 when the function is made (through its float64 value);
// every operation gives the correctly rounded binary32 result of its exact value on binary32
// operands, following the tree the grammar gives.  Results do not depend on the order in which
// independent subtrees are evaluated (operations are pure), so the compiler below picks that
// order to need few registers.
//
// An expression becomes a register program of the streaming kernel: in-place unary operations
// (negate, abs, sqrt, exp, with a constant: add, multiply, divide, divide the constant), binary
// operations between registers and constant loads.  The interpreter runs it op by op; a kernel
// compiled at run time for the pass gets the same ops as constants, i.e. straight-line code.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "sg_runtime.h"

using namespace sg;

namespace sgrt {

namespace {

struct Parser {
    const char* s;
    size_t i = 0;
    std::vector<ExprNode>& out;
    std::string err;
    Parser(const char* text, std::vector<ExprNode>& o) : s(text), out(o) {}

    void ws() {
        while (s[i] == ' ' || s[i] == '\t' || s[i] == '\n' || s[i] == '\r') ++i;
    }
    int add(ExprNode n) {
        out.push_back(n);
        return (int)out.size() - 1;
    }
    bool fail_at(const std::string& what) {
        if (err.empty()) err = what + " at offset " + std::to_string(i);
        return false;
    }
    bool accept(char c) {
        ws();
        if (s[i] == c) { ++i; return true; }
        return false;
    }
    bool expr(int* r) {
        int a;
        if (!term(&a)) return false;
        for (;;) {
            char op;
            if (accept('+')) op = '+';
            else if (accept('-')) op = '-';
            else break;
            int b;
            if (!term(&b)) return false;
            a = add({op == '+' ? (uint8_t)EX_ADD : (uint8_t)EX_SUB, 0.f, a, b});
        }
        *r = a;
        return true;
    }
    bool term(int* r) {
        int a;
        if (!unary(&a)) return false;
        for (;;) {
            char op;
            if (accept('*')) op = '*';
            else if (accept('/')) op = '/';
            else break;
            int b;
            if (!unary(&b)) return false;
            a = add({op == '*' ? (uint8_t)EX_MUL : (uint8_t)EX_DIV, 0.f, a, b});
        }
        *r = a;
        return true;
    }
    bool unary(int* r) {
        if (accept('-')) {
            int a;
            if (!unary(&a)) return false;
            *r = add({(uint8_t)EX_NEG, 0.f, a, -1});
            return true;
        }
        return primary(r);
    }
    bool primary(int* r) {
        ws();
        const char c = s[i];
        if ((c >= '0' && c <= '9') || c == '.') {
            // digits, an optional fraction, an optional exponent (no sign before the number:
            // that is unary minus)
            size_t j = i;
            while (s[j] >= '0' && s[j] <= '9') ++j;
            if (s[j] == '.') {
                ++j;
                while (s[j] >= '0' && s[j] <= '9') ++j;
            }
            if (j == i + 1 && s[i] == '.') return fail_at("a lone '.'");
            if (s[j] == 'e' || s[j] == 'E') {
                size_t k = j + 1;
                if (s[k] == '+' || s[k] == '-') ++k;
                if (s[k] >= '0' && s[k] <= '9') {
                    while (s[k] >= '0' && s[k] <= '9') ++k;
                    j = k;
                }
            }
            const std::string lit(s + i, j - i);
            i = j;
            // the literal's float64 value, rounded to binary32
            *r = add({(uint8_t)EX_CONST, (float)std::strtod(lit.c_str(), nullptr), -1, -1});
            return true;
        }
        if ((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || c == '_') {
            size_t j = i;
            while ((s[j] >= 'a' && s[j] <= 'z') || (s[j] >= 'A' && s[j] <= 'Z') || s[j] == '_') ++j;
            const std::string name(s + i, j - i);
            i = j;
            if (name == "x") {
                *r = add({(uint8_t)EX_X, 0.f, -1, -1});
                return true;
            }
            uint8_t k;
            if (name == "sqrt") k = EX_SQRT;
            else if (name == "abs") k = EX_ABS;
            else if (name == "exp") k = EX_EXP;
            else return fail_at("unknown name '" + name + "'");
            if (!accept('(')) return fail_at("expected '(' after " + name);
            int a;
            if (!expr(&a)) return false;
            if (!accept(')')) return fail_at("expected ')'");
            *r = add({k, 0.f, a, -1});
            return true;
        }
        if (accept('(')) {
            if (!expr(r)) return false;
            if (!accept(')')) return fail_at("expected ')'");
            return true;
        }
        return fail_at(c ? std::string("unexpected '") + c + "'" : std::string("unexpected end"));
    }
};

bool is_binary(uint8_t k) { return k == EX_ADD || k == EX_SUB || k == EX_MUL || k == EX_DIV; }

// Registers needed to evaluate node k into a given register without touching x's register
// (Sethi-Ullman numbering; a constant or x operand of a binary node costs nothing extra).
int need(const std::vector<ExprNode>& e, int k) {
    const ExprNode& n = e[k];
    if (n.kind == EX_X || n.kind == EX_CONST) return 1;
    if (!is_binary(n.kind)) return need(e, n.a);
    const ExprNode &L = e[n.a], &R = e[n.b];
    if (R.kind == EX_X || R.kind == EX_CONST) return need(e, n.a);  // d = d op x, d = d op c
    if (L.kind == EX_CONST) return need(e, n.b);                     // d = c op d
    const int a = need(e, n.a), b = need(e, n.b);
    return a == b ? a + 1 : std::max(a, b);
}

struct Gen {
    const std::vector<ExprNode>& e;
    std::vector<SgOp>& prog;
    int xr;  // register holding x (never written)
    void op(uint8_t code, int a, int b = 0, float c = 0.f) {
        SgOp o{};
        o.code = code;
        o.a = (uint8_t)a;
        o.dst = (uint8_t)a;
        o.b = (uint8_t)b;
        o.c0.f = c;
        prog.push_back(o);
    }
    void mov(int dst, int src) {
        if (dst == src) return;
        SgOp o{};
        o.code = MOV;
        o.a = (uint8_t)src;
        o.dst = (uint8_t)dst;
        prog.push_back(o);
    }
    // evaluate node k into register d using the free registers `fr` (none of them d or xr)
    bool gen(int k, int d, std::vector<int> fr) {
        const ExprNode& n = e[k];
        switch (n.kind) {
            case EX_X: mov(d, xr); return true;
            case EX_CONST: op(F_CONST, d, 0, n.c); return true;
            case EX_NEG: if (!gen(n.a, d, fr)) return false; op(F_NEG, d); return true;
            case EX_ABS: if (!gen(n.a, d, fr)) return false; op(F_ABS, d); return true;
            case EX_SQRT: if (!gen(n.a, d, fr)) return false; op(F_SQRT, d); return true;
            case EX_EXP: if (!gen(n.a, d, fr)) return false; op(F_EXP, d); return true;
            default: break;
        }
        const ExprNode &L = e[n.a], &R = e[n.b];
        const uint8_t bin = n.kind == EX_ADD ? F_ADD : n.kind == EX_SUB ? F_SUB : n.kind == EX_MUL ? F_MUL : F_DIV;
        if (R.kind == EX_CONST) {  // l op c: x - c is x + (-c) exactly
            if (!gen(n.a, d, fr)) return false;
            if (n.kind == EX_ADD) op(F_ADDC, d, 0, R.c);
            else if (n.kind == EX_SUB) op(F_ADDC, d, 0, -R.c);
            else if (n.kind == EX_MUL) op(F_MULC, d, 0, R.c);
            else op(F_DIVC, d, 0, R.c);
            return true;
        }
        if (L.kind == EX_CONST) {  // c op r: c + r and c * r commute exactly, c - r = (-r) + c
            if (!gen(n.b, d, fr)) return false;
            if (n.kind == EX_ADD) op(F_ADDC, d, 0, L.c);
            else if (n.kind == EX_SUB) { op(F_NEG, d); op(F_ADDC, d, 0, L.c); }
            else if (n.kind == EX_MUL) op(F_MULC, d, 0, L.c);
            else op(F_RDIVC, d, 0, L.c);
            return true;
        }
        if (R.kind == EX_X) {
            if (!gen(n.a, d, fr)) return false;
            op(bin, d, xr);
            return true;
        }
        // the subtree that needs more registers first, with every free register; then the
        // other into t = a free register, without it (Sethi-Ullman order)
        if (fr.empty()) return false;
        const int t = fr.back();
        std::vector<int> rest(fr.begin(), fr.end() - 1);
        if (need(e, n.a) >= need(e, n.b)) {
            if (!gen(n.a, d, fr) || !gen(n.b, t, rest)) return false;
        } else {
            std::vector<int> with_d = rest;
            with_d.push_back(d);  // d holds nothing yet
            if (!gen(n.b, t, with_d) || !gen(n.a, d, rest)) return false;
        }
        op(bin, d, t);  // d = d op t
        return true;
    }
};

}  // namespace

bool parse_expr(const char* text, std::vector<ExprNode>& out, int* root, std::string* why) {
    out.clear();
    Parser p(text, out);
    int r = -1;
    if (!p.expr(&r)) {
        *why = p.err;
        return false;
    }
    p.ws();
    if (p.s[p.i] != '\0') {
        *why = "unexpected '" + std::string(1, p.s[p.i]) + "' at offset " + std::to_string(p.i) + " after the expression";
        return false;
    }
    if (out.size() > 4096) {
        *why = "expression too long (more than 4096 nodes)";
        return false;
    }
    *root = r;
    return true;
}

int expr_temps(const std::vector<ExprNode>& e, int root) {
    // besides the map's own register: one for x, and need - 1 for intermediate values
    return need(e, root);
}

bool emit_expr(std::vector<SgOp>& prog, const std::vector<ExprNode>& e, int root, int r, const std::vector<int>& temps) {
    // x lives in r on entry and the result must end in r: x moves to a temporary first, so the
    // evaluation can overwrite r
    if (temps.empty()) return false;
    const int xr = temps.back();
    std::vector<int> fr(temps.begin(), temps.end() - 1);
    Gen g{e, prog, xr};
    g.mov(xr, r);
    return g.gen(root, r, fr);
}

}  // namespace sgrt

using namespace sgrt;

extern "C" sg_status sg_fn_expr(const char* text, sg_fn* out) {
    if (!text || !out) return fail(nullptr, SG_E_INVALID, "fn_expr: NULL argument");
    auto* nodes = new std::vector<ExprNode>();
    int root = -1;
    std::string why;
    if (!parse_expr(text, *nodes, &root, &why)) {
        delete nodes;
        return fail(nullptr, SG_E_INVALID, "fn_expr: " + why);
    }
    auto* fn = new sg_fn_s();
    fn->kind = FK_EXPR;
    fn->expr = nodes;
    fn->expr_root = root;
    *out = fn;
    return SG_OK;
}
