// gp_host.cpp -- host side of the library: status text, population
// generation (Sec. II-A, Sec. III-A) and population validation.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gp_internal.h"

namespace gp {

static thread_local std::string g_last_error;

gp_status fail(gp_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}
gp_status ok() { return GP_OK; }

namespace {

// Draw source for one program: words of Philox4x32-10 with counter
// (block, program, 0, kStreamInit), consumed in order.
class Draws {
  public:
    Draws(uint64_t seed, uint32_t item, uint32_t gen, uint32_t tag)
        : seed_(seed), item_(item), gen_(gen), tag_(tag) {}
    uint32_t next() {
        if ((n_ & 3u) == 0) blk_ = philox4x32_10(n_ >> 2, item_, gen_, tag_, seed_);
        return blk_.v[n_++ & 3u];
    }

  private:
    uint64_t seed_;
    uint32_t item_, gen_, tag_;
    uint32_t n_ = 0;
    Philox4 blk_{};
};

struct FuncSet {
    std::vector<uint32_t> all, unary, binary;
};

struct Gen {
    const gp_init_params& prm;
    FuncSet fs;
    bool consts_enabled;
    // output of the current program
    std::vector<uint32_t> nodes;
    std::vector<float> consts;

    explicit Gen(const gp_init_params& p) : prm(p) {
        for (uint32_t op = GP_OP_ADD; op < GP_OP_COUNT; ++op) {
            if (!(p.function_mask & (1u << op))) continue;
            fs.all.push_back(op);
            (arity(op) == 1 ? fs.unary : fs.binary).push_back(op);
        }
        consts_enabled = !(p.const_lo > p.const_hi);
    }

    bool const_available(int used) const {
        return consts_enabled && (prm.max_consts <= 0 || used < prm.max_consts);
    }

    float draw_const(Draws& dr) const {
        const float u = unit(dr.next());
        const float span = prm.const_hi - prm.const_lo;
        const float scaled = span * u;
        return prm.const_lo + scaled;
    }

    // Full / Grow: iterative pre-order walk with a stack of pending node depths.
    void tree(Draws& dr, int target_depth, bool full) {
        std::vector<int> pending{0};
        int used = 0;
        const int nf = prm.n_features;
        while (!pending.empty()) {
            const int depth = pending.back();
            pending.pop_back();
            const int n_term = nf + (const_available(used) ? 1 : 0);
            int pick;
            bool func;
            if (depth == target_depth) {
                func = false;
                pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(n_term)));
            } else if (depth == 0 || full) {
                func = true;
                pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(fs.all.size())));
            } else {
                const int nall = static_cast<int>(fs.all.size()) + n_term;
                pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(nall)));
                func = pick < static_cast<int>(fs.all.size());
                if (!func) pick -= static_cast<int>(fs.all.size());
            }
            if (func) {
                const uint32_t op = fs.all[pick];
                nodes.push_back(GP_NODE(op, 0));
                for (int a = 0; a < arity(op); ++a) pending.push_back(depth + 1);
            } else if (pick < nf) {
                nodes.push_back(GP_NODE(GP_OP_VAR, pick));
            } else {
                nodes.push_back(GP_NODE(GP_OP_CONST, used));
                consts.push_back(draw_const(dr));
                ++used;
            }
        }
    }

    // Exact length: fill positions right to left keeping the stack height h
    // reachable to exactly one value at position 0.
    void exact(Draws& dr) {
        uint32_t L = static_cast<uint32_t>(prm.min_len) +
                     below(dr.next(), static_cast<uint32_t>(prm.max_len - prm.min_len + 1));
        const bool no_unary = fs.unary.empty();
        if (no_unary && (L % 2u) == 0u) L = (L - 1 >= static_cast<uint32_t>(prm.min_len) && L > 1) ? L - 1 : L + 1;
        std::vector<uint32_t> rev;   // nodes in generation (right-to-left) order
        std::vector<float> cvals;    // constants in generation order
        rev.reserve(L);
        int h = 0;
        const int nf = prm.n_features;
        for (int i = static_cast<int>(L) - 1; i >= 0; --i) {
            const int n_term = nf + (const_available(static_cast<int>(cvals.size())) ? 1 : 0);
            bool t_ok = h + 1 <= GP_MAX_STACK && h <= i;
            bool u_ok = !no_unary && h >= 1 && h - 1 <= i;
            bool b_ok = !fs.binary.empty() && h >= 2 && h - 2 <= i;
            if (no_unary) {
                // only +1 / -1 steps remain: the height after this position
                // and the positions left must reach 1 together
                if (t_ok && ((h + i) & 1)) t_ok = false;
                if (b_ok && ((h - 2 + i) & 1)) b_ok = false;
            }
            const int nt = t_ok ? n_term : 0;
            const int nu = u_ok ? static_cast<int>(fs.unary.size()) : 0;
            const int nb = b_ok ? static_cast<int>(fs.binary.size()) : 0;
            int pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(nt + nu + nb)));
            if (pick < nt) {
                if (pick < nf) {
                    rev.push_back(GP_NODE(GP_OP_VAR, pick));
                } else {
                    rev.push_back(GP_NODE(GP_OP_CONST, 0));
                    cvals.push_back(draw_const(dr));
                }
                ++h;
            } else if ((pick -= nt) < nu) {
                rev.push_back(GP_NODE(fs.unary[pick], 0));
            } else {
                rev.push_back(GP_NODE(fs.binary[pick - nu], 0));
                --h;
            }
        }
        // emit in prefix order, numbering constants left to right
        size_t ci = cvals.size();
        uint32_t slot = 0;
        for (size_t k = rev.size(); k-- > 0;) {
            const uint32_t w = rev[k];
            if (GP_NODE_OP(w) == GP_OP_CONST) {
                nodes.push_back(GP_NODE(GP_OP_CONST, slot++));
                consts.push_back(cvals[--ci]);
            } else {
                nodes.push_back(w);
            }
        }
    }
};

}  // namespace
}  // namespace gp

using namespace gp;

extern "C" {

const char* gp_last_error(void) { return g_last_error.c_str(); }

const char* gp_version(void) { return "gp-mi355x 0.1 (gfx950)"; }

int gp_metric_larger_is_better(gp_metric metric) {
    switch (metric) {
    case GP_METRIC_MAE: case GP_METRIC_MSE: case GP_METRIC_RMSE: case GP_METRIC_LOGLOSS:
        return 0;
    case GP_METRIC_PEARSON: case GP_METRIC_SPEARMAN:
        return 1;
    default:
        return -1;
    }
}

gp_status gp_build_population(const gp_init_params* prm, uint32_t* nodes, int64_t nodes_cap,
                              int64_t* prog_off, float* consts, int64_t consts_cap,
                              int64_t* const_off, int32_t* len, int64_t* total_nodes,
                              int64_t* total_consts) {
    if (!prm) return fail(GP_ERR_INVALID_ARG, "gp_build_population: params is NULL");
    const gp_init_params& p = *prm;
    if (p.n_programs < 0 || p.n_features < 1)
        return fail(GP_ERR_INVALID_ARG, "gp_build_population: need n_programs >= 0 and n_features >= 1");
    const uint32_t allowed = ((1u << GP_OP_COUNT) - 1u) & ~3u;
    if (p.function_mask == 0 || (p.function_mask & ~allowed))
        return fail(GP_ERR_INVALID_ARG, "gp_build_population: function_mask must select functions (bits 2..11) only");
    if (p.method == GP_INIT_EXACT_LEN) {
        if (p.min_len < 1 || p.max_len < p.min_len || p.max_len > (1 << 20))
            return fail(GP_ERR_INVALID_ARG, "gp_build_population: need 1 <= min_len <= max_len <= 2^20");
        bool has_binary = false;
        for (uint32_t op = GP_OP_ADD; op <= GP_OP_DIV; ++op) has_binary |= (p.function_mask >> op) & 1u;
        if (!has_binary && p.max_len > 1)
            return fail(GP_ERR_INVALID_ARG, "gp_build_population: exact lengths above 1 need a binary function");
    } else if (p.method >= GP_INIT_RHH && p.method <= GP_INIT_GROW) {
        if (p.min_depth < 0 || p.max_depth < p.min_depth || p.max_depth > GP_MAX_STACK - 1)
            return fail(GP_ERR_INVALID_ARG, "gp_build_population: need 0 <= min_depth <= max_depth <= 19");
    } else {
        return fail(GP_ERR_INVALID_ARG, "gp_build_population: unknown method");
    }
    if (nodes && (!prog_off || !const_off || !len || (consts_cap > 0 && !consts)))
        return fail(GP_ERR_INVALID_ARG, "gp_build_population: output arrays must be given with nodes");

    Gen gen(p);
    int64_t n_nodes = 0, n_consts = 0;
    bool short_buf = false;
    for (int32_t prog = 0; prog < p.n_programs; ++prog) {
        Draws dr(p.seed, static_cast<uint32_t>(prog), 0u, kStreamInit);
        gen.nodes.clear();
        gen.consts.clear();
        if (p.method == GP_INIT_EXACT_LEN) {
            gen.exact(dr);
        } else {
            bool full;
            if (p.method == GP_INIT_RHH) full = !(unit(dr.next()) < 0.5f);
            else full = (p.method == GP_INIT_FULL);
            const int depth = p.min_depth +
                              static_cast<int>(below(dr.next(), static_cast<uint32_t>(p.max_depth - p.min_depth + 1)));
            gen.tree(dr, depth, full);
        }
        if (nodes) {
            prog_off[prog] = n_nodes;
            const_off[prog] = n_consts;
            len[prog] = static_cast<int32_t>(gen.nodes.size());
            if (n_nodes + static_cast<int64_t>(gen.nodes.size()) > nodes_cap ||
                n_consts + static_cast<int64_t>(gen.consts.size()) > consts_cap) {
                short_buf = true;
            } else {
                std::memcpy(nodes + n_nodes, gen.nodes.data(), gen.nodes.size() * sizeof(uint32_t));
                if (!gen.consts.empty())
                    std::memcpy(consts + n_consts, gen.consts.data(), gen.consts.size() * sizeof(float));
            }
        }
        n_nodes += static_cast<int64_t>(gen.nodes.size());
        n_consts += static_cast<int64_t>(gen.consts.size());
    }
    if (nodes) {
        prog_off[p.n_programs] = n_nodes;
        const_off[p.n_programs] = n_consts;
    }
    if (total_nodes) *total_nodes = n_nodes;
    if (total_consts) *total_consts = n_consts;
    if (short_buf)
        return fail(GP_ERR_BUFFER_TOO_SMALL, "gp_build_population: nodes_cap or consts_cap too small");
    return ok();
}

gp_status gp_validate_population(const uint32_t* nodes, const int64_t* prog_off,
                                 const int64_t* const_off, int32_t n_programs, int32_t n_features,
                                 int32_t* max_height, int32_t* bad_program) {
    if (n_programs < 0 || n_features < 1 || !prog_off || !const_off || (n_programs > 0 && !nodes))
        return fail(GP_ERR_INVALID_ARG, "gp_validate_population: bad arguments");
    for (int32_t p = 0; p < n_programs; ++p) {
        const int64_t a = prog_off[p], b = prog_off[p + 1];
        const int64_t nc = const_off[p + 1] - const_off[p];
        char buf[160];
        auto bad = [&](gp_status st, const char* why) {
            if (bad_program) *bad_program = p;
            std::snprintf(buf, sizeof buf, "gp_validate_population: program %d: %s", p, why);
            return fail(st, buf);
        };
        if (b <= a) return bad(GP_ERR_INVALID_PROGRAM, "empty program");
        if (nc < 0) return bad(GP_ERR_INVALID_PROGRAM, "negative constant count");
        int h = 0, hmax = 0;
        for (int64_t i = b - 1; i >= a; --i) {
            const uint32_t w = nodes[i];
            const uint32_t op = GP_NODE_OP(w);
            const int ar = arity(op);
            if (ar < 0) return bad(GP_ERR_INVALID_PROGRAM, "unknown opcode");
            if (op == GP_OP_VAR && GP_NODE_ARG(w) >= static_cast<uint32_t>(n_features))
                return bad(GP_ERR_INVALID_PROGRAM, "feature index out of range");
            if (op == GP_OP_CONST && static_cast<int64_t>(GP_NODE_ARG(w)) >= nc)
                return bad(GP_ERR_INVALID_PROGRAM, "constant slot out of range");
            if (h < ar) return bad(GP_ERR_INVALID_PROGRAM, "a function lacks operands");
            h += 1 - ar;
            if (h > GP_MAX_STACK) return bad(GP_ERR_STACK_OVERFLOW, "stack height above 20");
            if (h > hmax) hmax = h;
        }
        if (h != 1) return bad(GP_ERR_INVALID_PROGRAM, "more than one value left on the stack");
        if (max_height) max_height[p] = hmax;
    }
    return ok();
}

}  // extern "C"
