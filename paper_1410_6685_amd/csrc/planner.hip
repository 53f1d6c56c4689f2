// Planner: program (roots + contracts) -> passes of the streaming kernel, matrix products
// and product checks, in dependency order.
//
// The optimizer of Section 5 walks the execution-plan DAG and merges kernel vertices.
// Here the merge is a union-find over the element-wise nodes: a node joins the pass of each
// operand it does not read from memory.  Materialized nodes (roots, matrix-product
// operands) are written by the pass that computes them; "cut" nodes (fusion split points,
// operands of sortedness checks, every node when fusion is off) are in addition read back
// from memory by their consumers, which start a new pass.
// Inside a pass, filters become nested index spaces, and one filtered space per pass may be
// compacted (its ranks are what a materialized filter output and the index of a contract
// on that space need); a second such space makes the planner split before its filter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <map>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "sg_kernels.h"
#include "sg_runtime.h"

using namespace sg;

namespace sgrt {

namespace {

struct DSU {
    std::vector<int> p;
    int add() { p.push_back((int)p.size()); return (int)p.size() - 1; }
    int f(int x) { while (p[x] != x) x = p[x] = p[p[x]]; return x; }
    void u(int a, int b) { a = f(a); b = f(b); if (a != b) p[b] = a; }
};

bool is_source_node(const sg_node_s* n, const std::set<sg_node_s*>& mat) {
    return n->op == OPN_INPUT || is_kernel_node(n) || mat.count(const_cast<sg_node_s*>(n)) > 0;
}

bool active_contract(const Contract& c, sg_mode mode) {
    if (mode == SG_MODE_OFF) return false;
    if (c.kind == SG_REQUIRE) return true;
    return mode == SG_MODE_PRE_POST;
}

void need(std::set<sg_node_s*>& needed, sg_node_s* n) {
    if (!n || needed.count(n)) return;
    needed.insert(n);
    need(needed, n->src[0]);
    need(needed, n->src[1]);
}

}  // namespace

sg_status build_plan(sg_program_s* P, Plan* plan) {
    sg_ctx_s* ctx = P->ctx;
    const bool fused = ctx->fused;
    *plan = Plan();
    plan->generation = ctx->generation;
    for (int i = 0; i < (int)P->contracts.size(); ++i)
        if (active_contract(P->contracts[i], ctx->mode)) plan->active.push_back(i);

    std::set<sg_node_s*> needed;
    for (auto* r : P->roots) need(needed, r);
    for (int ci : plan->active) {
        const Contract& c = P->contracts[ci];
        need(needed, c.node);
        need(needed, c.a);
        need(needed, c.b);
        need(needed, c.r);
    }

    // ---- materialized set and cut set ------------------------------------------------------
    // mat: written to memory; cut: consumers read it from memory in a later pass
    std::set<sg_node_s*> mat, cut;
    for (auto* r : P->roots)
        if (is_collection(r) && r->op != OPN_INPUT && !is_kernel_node(r)) mat.insert(r);
    for (auto* s : P->splits)
        if (needed.count(s) && is_collection(s) && is_elementwise(s)) { mat.insert(s); cut.insert(s); }
    if (P->plan_split && needed.count(P->plan_split) && is_collection(P->plan_split) && is_elementwise(P->plan_split)) {
        mat.insert(P->plan_split);
        cut.insert(P->plan_split);
    }
    for (auto* n : needed) {
        if (is_kernel_node(n)) {  // its step reads its operands from memory
            for (auto* o : n->src)
                if (o && is_elementwise(o)) mat.insert(o);
        }
        if (!fused && is_elementwise(n) && is_collection(n)) { mat.insert(n); cut.insert(n); }
    }
    for (int ci : plan->active) {
        const Contract& c = P->contracts[ci];
        if (c.check == SG_CHECK_SORTED && is_elementwise(c.node)) { mat.insert(c.node); cut.insert(c.node); }
        if (c.check == SG_CHECK_PRODUCT) {
            for (auto* o : {c.node, c.a, c.b, c.r})
                if (is_elementwise(o)) mat.insert(o);
        }
        if (c.check == SG_CHECK_CLOSE && (c.node->op != OPN_REDUCE || c.node->red != SG_SUM || c.node->dtype != SG_F32))
            return fail(ctx, SG_E_INVALID, "close contract needs a float sum node");
    }
    // a quotient check reads the division's operands with its result: when the result is read
    // back from memory, so are they
    for (int ci : plan->active) {
        const Contract& c = P->contracts[ci];
        if (c.check != SG_CHECK_QUOTIENT || !cut.count(c.node)) continue;
        for (auto* x : {c.a, c.b})
            if (is_elementwise(x)) { mat.insert(x); cut.insert(x); }
    }

    // ---- passes ------------------------------------------------------------------------
    // Element-wise nodes joined by register operands form one pass each.  Passes that read a
    // common collection, or that read only input collections of one length, then share one
    // pass (each input is read once) unless one of them reads what the other writes, their
    // index spaces differ, or the joint pass would exceed the kernel's limits (then the plan
    // is rebuilt without sharing).
    bool hmerge = fused;
    for (int attempt = 0; attempt < 64; ++attempt) {
        DSU dsu;
        std::map<sg_node_s*, int> vnode;                          // compute vertex of a node
        std::map<std::pair<sg_node_s*, long>, int> vsrc;          // source vertex (node, consumer key)
        std::vector<sg_node_s*> elem;                             // needed element-wise nodes, id order
        for (auto* n : needed)
            if (is_elementwise(n)) elem.push_back(n);
        std::sort(elem.begin(), elem.end(), [](sg_node_s* a, sg_node_s* b) { return a->id < b->id; });
        for (auto* n : elem) vnode[n] = dsu.add();
        auto src_vertex = [&](sg_node_s* o, long key) {
            auto k = std::make_pair(o, key);
            auto it = vsrc.find(k);
            if (it != vsrc.end()) return it->second;
            int v = dsu.add();
            vsrc[k] = v;
            return v;
        };
        for (auto* n : elem) {
            for (auto* o : n->src) {
                if (!o) continue;
                if (is_source_node(o, cut)) dsu.u(vnode[n], src_vertex(o, (long)n->id));
                else dsu.u(vnode[n], vnode[o]);
            }
        }
        // contracts evaluated inside passes
        std::map<int, int> vcontract;  // contract -> vertex
        for (int ci : plan->active) {
            const Contract& c = P->contracts[ci];
            if (c.check == SG_CHECK_PRODUCT || c.check == SG_CHECK_COUNT_EQ) continue;  // not in a pass
            int v = dsu.add();
            vcontract[ci] = v;
            sg_node_s* t = c.node;
            if (c.check == SG_CHECK_CLOSE) { dsu.u(vnode[t], v); continue; }
            if (is_source_node(t, cut)) dsu.u(src_vertex(t, -1 - ci), v);
            else dsu.u(vnode[t], v);
            if (c.check == SG_CHECK_QUOTIENT) {  // the operands are read in the same pass
                for (auto* x : {c.a, c.b}) {
                    if (is_source_node(x, cut)) dsu.u(src_vertex(x, -1 - ci), v);
                    else dsu.u(vnode[x], v);
                }
            }
        }
        // group by component
        std::map<int, std::vector<sg_node_s*>> comp_nodes;
        std::map<int, std::vector<sg_node_s*>> comp_srcs;
        std::map<int, std::vector<int>> comp_contracts;
        for (auto* n : elem) comp_nodes[dsu.f(vnode[n])].push_back(n);
        for (auto& kv : vsrc) comp_srcs[dsu.f(kv.second)].push_back(kv.first.first);
        for (auto& kv : vcontract) comp_contracts[dsu.f(kv.second)].push_back(kv.first);
        std::set<int> roots_set;
        for (auto& kv : comp_nodes) roots_set.insert(kv.first);
        for (auto& kv : comp_contracts) roots_set.insert(kv.first);
        if (hmerge) {
            std::vector<int> roots(roots_set.begin(), roots_set.end());
            auto unique_srcs = [&](int r) {
                std::vector<sg_node_s*> v = comp_srcs[r];
                std::sort(v.begin(), v.end());
                v.erase(std::unique(v.begin(), v.end()), v.end());
                return v;
            };
            // producer component of every node computed in a pass
            std::map<sg_node_s*, int> comp_of;
            for (int r : roots)
                for (auto* x : comp_nodes[r]) comp_of[x] = r;
            // is `x` (a pass source) written by component `from`, directly or through products?
            std::function<bool(sg_node_s*, int)> made_in = [&](sg_node_s* x, int from) {
                if (!x) return false;
                auto it = comp_of.find(x);
                if (it != comp_of.end()) return it->second == from;
                if (is_kernel_node(x)) return made_in(x->src[0], from) || made_in(x->src[1], from);
                return false;
            };
            // does component `to` read (transitively) what component `from` writes?
            std::function<bool(int, int, std::set<int>&)> reaches = [&](int from, int to, std::set<int>& seen) {
                if (from == to) return true;
                if (!seen.insert(from).second) return false;
                for (int r : roots) {
                    if (r == from) continue;
                    for (auto* x : unique_srcs(r))
                        if (made_in(x, from) && reaches(r, to, seen)) return true;
                }
                return false;
            };
            auto compatible = [&](int a, int b) {
                std::vector<sg_node_s*> all = unique_srcs(a), sb = unique_srcs(b);
                if (all.empty() || sb.empty()) return false;
                bool shared = false, inputs_only = true;
                for (auto* x : sb) shared |= std::find(all.begin(), all.end(), x) != all.end();
                all.insert(all.end(), sb.begin(), sb.end());
                std::sort(all.begin(), all.end());
                all.erase(std::unique(all.begin(), all.end()), all.end());
                if ((int)all.size() > MAX_IN) return false;
                sg_node_s* s0 = all[0];
                for (auto* x : all) {
                    inputs_only &= x->op == OPN_INPUT;
                    if (x->n != s0->n) return false;
                    const bool cx = x->space != 0, c0 = s0->space != 0;  // compacted collections
                    if (cx != c0 || (cx && x != s0 && x->space != s0->space)) return false;
                }
                if (!shared && !inputs_only) return false;
                std::set<int> s1, s2;
                return !reaches(a, b, s1) && !reaches(b, a, s2);
            };
            for (bool merged = true; merged;) {
                merged = false;
                for (size_t i = 0; i < roots.size() && !merged; ++i)
                    for (size_t j = i + 1; j < roots.size() && !merged; ++j) {
                        const int a = roots[i], b = roots[j];
                        if (!compatible(a, b)) continue;
                        for (auto* x : comp_nodes[b]) {
                            comp_nodes[a].push_back(x);
                            comp_of[x] = a;
                        }
                        for (auto* x : comp_srcs[b]) comp_srcs[a].push_back(x);
                        for (int c : comp_contracts[b]) comp_contracts[a].push_back(c);
                        std::sort(comp_nodes[a].begin(), comp_nodes[a].end(),
                                  [](sg_node_s* x, sg_node_s* y) { return x->id < y->id; });
                        comp_nodes.erase(b);
                        comp_srcs.erase(b);
                        comp_contracts.erase(b);
                        roots.erase(roots.begin() + j);
                        merged = true;
                    }
            }
            roots_set = std::set<int>(roots.begin(), roots.end());
        }

        plan->insts.clear();
        plan->steps.clear();
        bool resplit = false;
        std::map<sg_node_s*, int> producer;  // materialized node -> pass index
        std::vector<std::vector<sg_node_s*>> inst_srcs;

        for (int root : roots_set) {
            std::vector<sg_node_s*> nodes = comp_nodes[root];
            std::vector<sg_node_s*> srcs = comp_srcs[root];
            std::vector<int> cons = comp_contracts[root];
            std::sort(srcs.begin(), srcs.end(), [](sg_node_s* a, sg_node_s* b) { return a->id < b->id; });
            srcs.erase(std::unique(srcs.begin(), srcs.end()), srcs.end());
            std::sort(cons.begin(), cons.end());
            if (srcs.empty()) return fail(ctx, SG_E_UNSUPPORTED, "a pass without a source collection");
            if ((int)srcs.size() > MAX_IN) return fail(ctx, SG_E_UNSUPPORTED, "a pass reads more than 4 source collections; add a split point");

            InstPlan ip;
            ip.sources = srcs;
            // element count: every source of a pass has the same index space
            sg_node_s* s0 = srcs[0];
            for (auto* s : srcs) {
                if (s->n != s0->n) return fail(ctx, SG_E_SHAPE, "sources of one pass differ in length");
                const bool cs = s->space != 0, c0 = s0->space != 0;  // compacted collections
                if (cs != c0 || (cs && s != s0 && s->space != s0->space))
                    return fail(ctx, SG_E_SHAPE, "sources of one pass lie in different index spaces");
            }
            ip.n = s0->n;
            ip.n_src = s0->space != 0 ? s0 : nullptr;  // count of a compacted source: on the device

            // index spaces: 0 = the sources' space; each filter in the pass opens a new one
            std::map<sg_node_s*, int> sp;
            for (auto* s : srcs) sp[s] = 0;
            std::map<int, sg_node_s*> space_filter;
            int nspace = 1;
            std::set<sg_node_s*> in_pass(nodes.begin(), nodes.end());
            auto space_of = [&](sg_node_s* x) -> int {
                auto it = sp.find(x);
                return it == sp.end() ? 0 : it->second;
            };
            for (auto* n : nodes) {
                if (n->op == OPN_FILTER) {
                    if (nspace >= MAX_SPACES && hmerge) {
                        hmerge = false;
                        resplit = true;
                        break;
                    }
                    if (nspace >= MAX_SPACES) {
                        // too many nested filters for one pass: the operands of this and every
                        // later filter of the pass are written out and read back by a new pass
                        bool cut_any = false;
                        bool past = false;
                        for (auto* f : nodes) {
                            past |= f == n;
                            if (!past || f->op != OPN_FILTER) continue;
                            sg_node_s* o = f->src[0];
                            if (o && is_elementwise(o) && is_collection(o) && !cut.count(o)) {
                                mat.insert(o);
                                cut.insert(o);
                                cut_any = true;
                            }
                        }
                        if (!cut_any) return fail(ctx, SG_E_UNSUPPORTED, "more than 7 filters in one pass; add a split point");
                        resplit = true;
                        break;
                    }
                    space_filter[nspace] = n;
                    sp[n] = nspace++;
                } else {
                    sp[n] = space_of(n->src[0]);
                }
            }
            if (resplit) break;
            // spaces whose ranks are needed
            std::set<int> scan_need;
            for (auto* n : nodes)
                if (mat.count(n) && sp[n] != 0) scan_need.insert(sp[n]);
            for (int ci : cons) {
                const Contract& c = P->contracts[ci];
                if ((c.check == SG_CHECK_FOR_ALL || c.check == SG_CHECK_EXISTS) && in_pass.count(c.node) && sp[c.node] != 0)
                    scan_need.insert(sp[c.node]);
            }
            if (scan_need.size() > 1 && hmerge) {
                hmerge = false;
                resplit = true;
                break;
            }
            if (scan_need.size() > 1) {
                // keep the first; split before the filter of every other one
                auto it = scan_need.begin();
                for (++it; it != scan_need.end(); ++it) {
                    sg_node_s* f = space_filter[*it];
                    mat.insert(f->src[0]);
                    cut.insert(f->src[0]);
                }
                resplit = true;
                break;
            }
            ip.scan_space = scan_need.empty() ? 0 : *scan_need.begin();

            // ---- register allocation and program emission -------------------------------
            // last use (position in `nodes`) of every value; contracts on sources use -1
            std::map<sg_node_s*, int> pos;
            for (int i = 0; i < (int)nodes.size(); ++i) pos[nodes[i]] = i;
            auto value_of = [&](sg_node_s* x) {  // the node whose register holds x's values
                while (x->op == OPN_FILTER && in_pass.count(x)) x = x->src[0];
                return x;
            };
            std::map<sg_node_s*, int> last;
            auto use = [&](sg_node_s* x, int at) {
                sg_node_s* v = value_of(x);
                auto it = last.find(v);
                if (it == last.end() || it->second < at) last[v] = at;
            };
            for (int i = 0; i < (int)nodes.size(); ++i)
                for (auto* o : nodes[i]->src)
                    if (o) use(o, i);
            for (int ci : cons) {
                const Contract& c = P->contracts[ci];
                if (c.check == SG_CHECK_CLOSE) {
                    use(c.node->src[0], pos[c.node]);
                } else if (in_pass.count(c.node)) {
                    use(c.node, pos[c.node]);
                    if (c.check == SG_CHECK_QUOTIENT) {  // operands live past the division
                        use(c.a, pos[c.node] + 1);
                        use(c.b, pos[c.node] + 1);
                    }
                } else {
                    use(c.node, -1);
                    if (c.check == SG_CHECK_QUOTIENT) {
                        use(c.a, -1);
                        use(c.b, -1);
                    }
                }
            }
            const int END = 1 << 30;
            for (auto* n : nodes)
                if (mat.count(n) && sp[n] != 0) use(n, END);  // compacted emits read registers after the scan

            int owner_last[NREG];
            sg_node_s* owner[NREG];
            for (int r = 0; r < NREG; ++r) { owner_last[r] = -2; owner[r] = nullptr; }
            std::map<sg_node_s*, int> reg;
            for (int k = 0; k < (int)srcs.size(); ++k) {
                reg[srcs[k]] = k;
                owner[k] = srcs[k];
                owner_last[k] = last.count(srcs[k]) ? last[srcs[k]] : -1;
            }
            auto free_dead = [&](int at) {
                for (int r = 0; r < NREG; ++r)
                    if (owner[r] && owner_last[r] <= at) { owner[r] = nullptr; owner_last[r] = -2; }
            };
            auto alloc = [&](sg_node_s* v) -> int {
                for (int r = 0; r < NREG; ++r)
                    if (!owner[r]) {
                        owner[r] = v;
                        owner_last[r] = last.count(v) ? last[v] : -1;
                        reg[v] = r;
                        return r;
                    }
                return -1;
            };
            auto reg_of = [&](sg_node_s* x) { return reg[value_of(x)]; };

            std::vector<SgOp>& prog = ip.prog;
            int nslots = 0;
            auto new_slot = [&](uint8_t kind) {
                ip.slot_kind.push_back(kind);
                return nslots++;
            };
            auto emit_check = [&](int ci, int r, int space, sg_dtype dt) {
                const Contract& c = P->contracts[ci];
                SgOp o{};
                if (c.check == SG_CHECK_SORTED) {
                    o.code = dt == SG_F32 ? CHK_SORTED_F : CHK_SORTED_I;
                    o.a = (uint8_t)r;
                    o.b = (uint8_t)r;  // sources sit in the register of their input index
                } else if (c.check == SG_CHECK_QUOTIENT) {
                    SgOp q{};
                    q.code = P_QUOT;
                    q.a = (uint8_t)r;
                    q.b = (uint8_t)reg_of(c.a);
                    q.dst = (uint8_t)reg_of(c.b);
                    prog.push_back(q);
                    o.code = CHK_ALL;
                    o.sp = (uint8_t)space;
                } else {
                    emit_pred(prog, c.pred, r, dt);
                    o.code = c.check == SG_CHECK_FOR_ALL ? CHK_ALL : CHK_ANY;
                    o.sp = (uint8_t)space;
                }
                o.aux = (uint8_t)new_slot(SLOT_MAX64);
                prog.push_back(o);
                ip.checks.push_back({ci, o.aux});
            };

            // contracts on sources come first
            for (int ci : cons) {
                const Contract& c = P->contracts[ci];
                if (c.check == SG_CHECK_CLOSE || in_pass.count(c.node)) continue;
                emit_check(ci, reg[c.node], 0, c.node->dtype);
            }
            free_dead(-1);
            bool too_many = false;
            int nemit_c = 0;
            for (int i = 0; i < (int)nodes.size() && !too_many; ++i) {
                sg_node_s* n = nodes[i];
                const int s_here = sp[n];
                switch (n->op) {
                    case OPN_MAP: {
                        sg_node_s* a = value_of(n->src[0]);
                        int ra = reg[a];
                        int rd;
                        if (owner_last[ra] <= i && !(owner[ra] && mat.count(owner[ra]) && sp[owner[ra]] != 0)) {
                            rd = ra;  // operand dies here: work in place
                            owner[ra] = n;
                            owner_last[ra] = last.count(n) ? last[n] : -1;
                            reg[n] = ra;
                        } else {
                            rd = alloc(n);
                            if (rd < 0) { too_many = true; break; }
                            SgOp mv{};
                            mv.code = MOV; mv.a = (uint8_t)ra; mv.dst = (uint8_t)rd;
                            prog.push_back(mv);
                        }
                        // registers free for the map's duration (expression agents use them)
                        std::vector<int> temps;
                        for (int r = 0; r < NREG && (int)temps.size() < fn_temps(n->fn); ++r)
                            if (!owner[r] && r != rd) temps.push_back(r);
                        if (!emit_fn(prog, n->fn, rd, n->src[0]->dtype, temps)) { too_many = true; break; }
                    } break;
                    case OPN_ZIP: {
                        int ra = reg_of(n->src[0]), rb = reg_of(n->src[1]);
                        const bool comm = n->binop == SG_ADD || n->binop == SG_MUL;
                        auto dies = [&](int r) {
                            return owner_last[r] <= i && !(owner[r] && mat.count(owner[r]) && sp[owner[r]] != 0);
                        };
                        int rd;
                        if (dies(ra) && ra != rb) {
                            rd = ra;
                        } else if (comm && dies(rb) && ra != rb) {
                            rd = rb;
                            std::swap(ra, rb);
                        } else {
                            rd = alloc(n);
                            if (rd < 0) { too_many = true; break; }
                            SgOp mv{};
                            mv.code = MOV; mv.a = (uint8_t)ra; mv.dst = (uint8_t)rd;
                            prog.push_back(mv);
                            ra = rd;
                        }
                        owner[rd] = n;
                        owner_last[rd] = last.count(n) ? last[n] : -1;
                        reg[n] = rd;
                        SgOp o{};
                        const bool f = n->dtype == SG_F32;
                        o.code = n->binop == SG_ADD   ? (f ? F_ADD : I_ADD)
                                 : n->binop == SG_SUB ? (f ? F_SUB : I_SUB)
                                 : n->binop == SG_MUL ? (f ? F_MUL : I_MUL)
                                                      : F_DIV;
                        o.a = (uint8_t)ra;
                        o.b = (uint8_t)rb;
                        o.dst = (uint8_t)ra;
                        prog.push_back(o);
                    } break;
                    case OPN_FILTER: {
                        int r = reg_of(n->src[0]);
                        emit_pred(prog, n->pred, r, n->dtype);
                        SgOp o{};
                        o.code = FILTER;
                        o.sp = (uint8_t)s_here;
                        o.sp2 = (uint8_t)space_of(n->src[0]);
                        prog.push_back(o);
                    } break;
                    case OPN_REDUCE: {
                        sg_node_s* src = n->src[0];
                        int r = reg_of(src);
                        const int ssp = space_of(src);
                        const bool f = src->dtype == SG_F32;
                        InstPlan::ScalarOut so{n, -1, -1, -1};
                        SgOp o{};
                        o.a = (uint8_t)r;
                        o.sp = (uint8_t)ssp;
                        switch (n->red) {
                            case SG_SUM: case SG_AVG:
                                if (f) {
                                    if (ip.nsum >= MAX_SUMS) { too_many = true; break; }
                                    o.code = RED_SUM_F; o.aux = (uint8_t)ip.nsum; so.sum = ip.nsum++;
                                } else {
                                    o.code = RED_SUM_I; o.aux = (uint8_t)new_slot(SLOT_ADD); so.slot = o.aux;
                                }
                                prog.push_back(o);
                                if (n->red == SG_AVG) {
                                    SgOp c{};
                                    c.code = RED_COUNT; c.sp = (uint8_t)ssp; c.aux = (uint8_t)new_slot(SLOT_ADD);
                                    so.count_slot = c.aux;
                                    prog.push_back(c);
                                }
                                break;
                            case SG_MAX: case SG_MIN:
                                o.code = n->red == SG_MAX ? (f ? RED_MAX_F : RED_MAX_I) : (f ? RED_MIN_F : RED_MIN_I);
                                o.aux = (uint8_t)new_slot(SLOT_MAX32);
                                so.slot = o.aux;
                                prog.push_back(o);
                                break;
                            case SG_COUNT:
                                o.code = RED_COUNT; o.aux = (uint8_t)new_slot(SLOT_ADD);
                                so.slot = o.aux;
                                prog.push_back(o);
                                break;
                        }
                        ip.scalars.push_back(so);
                        // close contracts on this sum: |x| sum when a relative tolerance is asked for
                        for (int ci : cons) {
                            const Contract& c = P->contracts[ci];
                            if (c.check != SG_CHECK_CLOSE || c.node != n || c.rel_tol == 0.0) continue;
                            if (ip.nsum >= MAX_SUMS) { too_many = true; break; }
                            SgOp a{};
                            a.code = RED_ABSSUM_F; a.a = (uint8_t)r; a.sp = (uint8_t)ssp; a.aux = (uint8_t)ip.nsum;
                            ip.abssums.push_back({ci, ip.nsum++});
                            prog.push_back(a);
                        }
                    } break;
                    default:
                        return fail(ctx, SG_E_INVALID, "planner: unexpected node in a pass");
                }
                if (too_many) break;
                // materialize
                if (mat.count(n)) {
                    if ((int)ip.outs.size() >= MAX_OUT) { too_many = true; break; }
                    SgOp o{};
                    o.code = EMIT;
                    o.a = (uint8_t)reg_of(n);
                    o.aux = (uint8_t)ip.outs.size();
                    o.sp = (uint8_t)s_here;
                    if (s_here != 0) {
                        if (s_here != ip.scan_space || nemit_c >= MAX_CEMIT) { too_many = true; break; }
                        ++nemit_c;
                        ip.compacted.push_back(n);
                    }
                    ip.outs.push_back(n);
                    prog.push_back(o);
                    producer[n] = (int)plan->insts.size();
                }
                // contracts on this node
                for (int ci : cons) {
                    const Contract& c = P->contracts[ci];
                    if (c.check == SG_CHECK_CLOSE || c.node != n) continue;
                    emit_check(ci, reg_of(n), s_here, n->dtype);
                }
                free_dead(i);
            }
            if (too_many && hmerge) {
                hmerge = false;
                resplit = true;
                break;
            }
            if (too_many) return fail(ctx, SG_E_UNSUPPORTED, "chain too large for one pass (registers, sums, outputs); add a split point");
            if (ip.scan_space != 0) {
                SgOp c{};
                c.code = RED_COUNT; c.sp = (uint8_t)ip.scan_space; c.aux = (uint8_t)new_slot(SLOT_ADD);
                ip.count_slot = c.aux;
                prog.push_back(c);
            }
            if (ip.n_src) {
                // dense outputs of a pass over a compacted source have its (device) count
                SgOp c{};
                c.code = RED_COUNT; c.sp = 0; c.aux = (uint8_t)new_slot(SLOT_ADD);
                ip.base_count_slot = c.aux;
                prog.push_back(c);
            }
            int ndefer = 0;
            for (auto& o : prog) ndefer += (o.code == CHK_ALL || o.code == CHK_ANY) && o.sp != 0 && o.sp == ip.scan_space;
            if (hmerge && ((int)prog.size() > MAX_INLINE_OPS || ndefer > MAX_DEFER || nslots > MAX_SLOTS)) {
                hmerge = false;
                resplit = true;
                break;
            }
            if ((int)prog.size() > MAX_INLINE_OPS) return fail(ctx, SG_E_UNSUPPORTED, "program longer than 48 operations; add a split point");
            if (ndefer > MAX_DEFER) return fail(ctx, SG_E_UNSUPPORTED, "more than 2 quantified contracts on a compacted collection in one pass");
            if (nslots > MAX_SLOTS) return fail(ctx, SG_E_UNSUPPORTED, "more than 16 reductions/contracts in one pass");
            ip.result_index = (int)plan->insts.size();
            plan->insts.push_back(ip);
            inst_srcs.push_back(srcs);
        }
        if (resplit) continue;

        // ---- steps in dependency order -------------------------------------------------
        std::vector<sg_node_s*> mm;  // kernel nodes: matrix products, sorts, concatenations
        for (auto* n : needed)
            if (is_kernel_node(n)) mm.push_back(n);
        std::sort(mm.begin(), mm.end(), [](sg_node_s* a, sg_node_s* b) { return a->id < b->id; });
        std::vector<int> prods;
        for (int ci : plan->active)
            if (P->contracts[ci].check == SG_CHECK_PRODUCT) prods.push_back(ci);
        // items: passes, products, checks; each waits for the producers of its sources
        const int NI = (int)plan->insts.size(), NM = (int)mm.size(), NP = (int)prods.size();
        std::vector<std::vector<sg_node_s*>> deps(NI + NM + NP);
        for (int i = 0; i < NI; ++i) deps[i] = inst_srcs[i];
        for (int j = 0; j < NM; ++j) {
            for (auto* o : mm[j]->src)
                if (o) deps[NI + j].push_back(o);
        }
        for (int k = 0; k < NP; ++k) {
            const Contract& c = P->contracts[prods[k]];
            deps[NI + NM + k] = {c.node, c.a, c.b, c.r};
        }
        std::map<sg_node_s*, int> made_by;  // node -> item
        for (auto& kv : producer) made_by[kv.first] = kv.second;
        for (int j = 0; j < NM; ++j) made_by[mm[j]] = NI + j;
        std::vector<int> done(NI + NM + NP, 0);
        int remaining = NI + NM + NP;
        while (remaining > 0) {
            bool progress = false;
            for (int it = 0; it < NI + NM + NP; ++it) {
                if (done[it]) continue;
                bool ready = true;
                for (auto* d : deps[it]) {
                    auto m = made_by.find(d);
                    if (m != made_by.end() && !done[m->second]) { ready = false; break; }
                }
                if (!ready) continue;
                Step st;
                if (it < NI) { st.kind = Step::STREAM; st.inst = it; }
                else if (it < NI + NM && mm[it - NI]->op == OPN_MATMUL) {
                    st.kind = Step::GEMM; st.A = mm[it - NI]->src[0]; st.B = mm[it - NI]->src[1]; st.C = mm[it - NI];
                } else if (it < NI + NM) {
                    st.kind = Step::NODE; st.node = mm[it - NI];
                }
                else {
                    const Contract& c = P->contracts[prods[it - NI - NM]];
                    st.kind = Step::PRODUCT; st.C = c.node; st.A = c.a; st.B = c.b; st.R = c.r; st.contract = prods[it - NI - NM];
                }
                plan->steps.push_back(st);
                done[it] = 1;
                --remaining;
                progress = true;
            }
            if (!progress) return fail(ctx, SG_E_INVALID, "planner: cyclic dependency");
        }
        plan->mats.assign(mat.begin(), mat.end());
        plan->valid = true;
        return SG_OK;
    }
    return fail(ctx, SG_E_UNSUPPORTED, "planner: could not place the filters (too many compacted spaces)");
}

}  // namespace sgrt
