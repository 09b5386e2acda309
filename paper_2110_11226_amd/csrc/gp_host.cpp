// gp_host.cpp -- host side of the library: status text, population
// generation (Sec. II-A, Sec. III-A) and population validation.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
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

// ---- user function registry (Sec. V: custom function sets) ----
static std::mutex g_user_mu;
static UserDefs g_user{};
static std::atomic<uint32_t> g_user_mask{0u};

void user_defs(UserDefs* out) {
    std::lock_guard<std::mutex> lk(g_user_mu);
    *out = g_user;
}
uint32_t user_defined_mask() { return g_user_mask.load(); }

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
        for (uint32_t op = GP_OP_ADD; op < GP_OP_LIMIT; ++op) {
            if (!(p.function_mask & (1u << op)) || arity(op) < 1) continue;
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

    // One program by the configured method (Sec. II-A): ramped half-and-half
    // draws Grow or Full and then the depth; exact length draws the length.
    void program(Draws& dr) {
        nodes.clear();
        consts.clear();
        if (prm.method == GP_INIT_EXACT_LEN) {
            exact(dr);
            return;
        }
        bool full;
        if (prm.method == GP_INIT_RHH) full = !(unit(dr.next()) < 0.5f);
        else full = (prm.method == GP_INIT_FULL);
        const int depth = prm.min_depth +
                          static_cast<int>(below(dr.next(), static_cast<uint32_t>(prm.max_depth - prm.min_depth + 1)));
        tree(dr, depth, full);
    }
};

gp_status check_init(const gp_init_params& p, const char* who) {
    if (p.n_programs < 0 || p.n_features < 1)
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": need n_programs >= 0 and n_features >= 1");
    if (p.function_mask == 0 || (p.function_mask & ~allowed_function_mask()))
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": function_mask must select functions (bits 2..22, "
                                                           "or 24..31 once defined) only");
    if (p.method == GP_INIT_EXACT_LEN) {
        if (p.min_len < 1 || p.max_len < p.min_len || p.max_len > (1 << 20))
            return fail(GP_ERR_INVALID_ARG, std::string(who) + ": need 1 <= min_len <= max_len <= 2^20");
        bool has_binary = false;
        for (uint32_t op = GP_OP_ADD; op < GP_OP_LIMIT; ++op) has_binary |= arity(op) == 2 && ((p.function_mask >> op) & 1u);
        if (!has_binary && p.max_len > 1)
            return fail(GP_ERR_INVALID_ARG, std::string(who) + ": exact lengths above 1 need a binary function");
    } else if (p.method >= GP_INIT_RHH && p.method <= GP_INIT_GROW) {
        if (p.min_depth < 0 || p.max_depth < p.min_depth || p.max_depth > GP_MAX_STACK - 1)
            return fail(GP_ERR_INVALID_ARG, std::string(who) + ": need 0 <= min_depth <= max_depth <= 19");
    } else {
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": unknown method");
    }
    return GP_OK;
}

// ---------------------------------------------------------------------------
// Genetic operations (Sec. II-A, Sec. III-C2), applied on the host.
// ---------------------------------------------------------------------------
// A program being assembled: node words, with each constant's value carried
// beside its node; slots are renumbered in prefix order when it is emitted.
struct Prog {
    std::vector<uint32_t> w;
    std::vector<float> val;
};

Prog load_prog(const uint32_t* nodes, const int64_t* prog_off, const float* consts, const int64_t* const_off,
               int32_t p) {
    Prog g;
    const float* pc = consts ? consts + const_off[p] : nullptr;
    for (int64_t i = prog_off[p]; i < prog_off[p + 1]; ++i) {
        const uint32_t w = nodes[i];
        g.w.push_back(w);
        g.val.push_back(GP_NODE_OP(w) == GP_OP_CONST ? pc[GP_NODE_ARG(w)] : 0.0f);
    }
    return g;
}

Prog from_gen(const Gen& gen) {
    Prog g;
    for (uint32_t w : gen.nodes) {
        g.w.push_back(w);
        g.val.push_back(GP_NODE_OP(w) == GP_OP_CONST ? gen.consts[GP_NODE_ARG(w)] : 0.0f);
    }
    return g;
}

// One past the last node of the subtree whose root is at position s.
size_t subtree_end(const std::vector<uint32_t>& w, size_t s) {
    int open = 1;
    size_t i = s;
    while (open > 0) {
        open += arity(GP_NODE_OP(w[i])) - 1;
        ++i;
    }
    return i;
}

// Peak stack height of the right-to-left scan of a valid program.
int peak_height(const std::vector<uint32_t>& w) {
    int h = 0, hmax = 0;
    for (size_t i = w.size(); i-- > 0;) {
        h += 1 - arity(GP_NODE_OP(w[i]));
        hmax = std::max(hmax, h);
    }
    return hmax;
}

// parent[0:s) + donor[ds:de) + parent[e:)
Prog splice(const Prog& p, size_t s, size_t e, const Prog& d, size_t ds, size_t de) {
    Prog c;
    c.w.assign(p.w.begin(), p.w.begin() + s);
    c.val.assign(p.val.begin(), p.val.begin() + s);
    c.w.insert(c.w.end(), d.w.begin() + ds, d.w.begin() + de);
    c.val.insert(c.val.end(), d.val.begin() + ds, d.val.begin() + de);
    c.w.insert(c.w.end(), p.w.begin() + e, p.w.end());
    c.val.insert(c.val.end(), p.val.begin() + e, p.val.end());
    return c;
}

// Crossover with hoisting (Sec. III-C2): a uniformly chosen subtree of the
// parent is replaced by a uniformly chosen subtree of the donor; while the
// child's stack would exceed GP_MAX_STACK or its length max_len, the donor
// subtree is replaced by a uniformly chosen proper subtree of itself.
Prog crossover(const Prog& parent, const Prog& donor, Draws& dr, int32_t max_len) {
    const size_t s = below(dr.next(), static_cast<uint32_t>(parent.w.size()));
    const size_t e = subtree_end(parent.w, s);
    size_t ds = below(dr.next(), static_cast<uint32_t>(donor.w.size()));
    size_t de = subtree_end(donor.w, ds);
    for (;;) {
        Prog c = splice(parent, s, e, donor, ds, de);
        const bool fits = peak_height(c.w) <= GP_MAX_STACK && static_cast<int64_t>(c.w.size()) <= max_len;
        if (fits || de - ds == 1) return c;
        ds = ds + 1 + below(dr.next(), static_cast<uint32_t>(de - ds - 1));
        de = subtree_end(donor.w, ds);
    }
}

// Hoist mutation: a uniformly chosen subtree is replaced by a uniformly
// chosen subtree of itself (possibly itself).
Prog hoist(const Prog& parent, Draws& dr) {
    const size_t s = below(dr.next(), static_cast<uint32_t>(parent.w.size()));
    const size_t e = subtree_end(parent.w, s);
    const size_t s2 = s + below(dr.next(), static_cast<uint32_t>(e - s));
    const size_t e2 = subtree_end(parent.w, s2);
    return splice(parent, s, e, parent, s2, e2);
}

// Point mutation: each node, in prefix order, is replaced with probability
// p_replace -- a function by one of the same arity from the function set, a
// terminal by a variable or (if constants are enabled and the program's
// other constants number below max_consts) a new constant.
Prog point(const Prog& parent, const Gen& gen, float p_replace, Draws& dr) {
    Prog c = parent;
    int n_const = 0;
    for (uint32_t w : c.w) n_const += GP_NODE_OP(w) == GP_OP_CONST;
    const int nf = gen.prm.n_features;
    for (size_t j = 0; j < c.w.size(); ++j) {
        if (!(unit(dr.next()) < p_replace)) continue;
        const uint32_t op = GP_NODE_OP(c.w[j]);
        const int ar = arity(op);
        if (ar > 0) {
            const std::vector<uint32_t>& set = ar == 1 ? gen.fs.unary : gen.fs.binary;
            if (set.empty()) continue;
            c.w[j] = GP_NODE(set[below(dr.next(), static_cast<uint32_t>(set.size()))], 0);
            continue;
        }
        const int others = n_const - (op == GP_OP_CONST ? 1 : 0);
        const int n_term = nf + (gen.const_available(others) ? 1 : 0);
        const int pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(n_term)));
        if (pick < nf) {
            c.w[j] = GP_NODE(GP_OP_VAR, pick);
            c.val[j] = 0.0f;
            n_const = others;
        } else {
            c.w[j] = GP_NODE(GP_OP_CONST, 0);
            c.val[j] = gen.draw_const(dr);
            n_const = others + 1;
        }
    }
    return c;
}

// float32 cumulative thresholds of the operation draw
struct OpThresholds {
    float t[4];
};
OpThresholds thresholds(const gp_evolve_params& e) {
    OpThresholds o;
    o.t[0] = e.p_crossover;
    o.t[1] = o.t[0] + e.p_subtree;
    o.t[2] = o.t[1] + e.p_hoist;
    o.t[3] = o.t[2] + e.p_point;
    return o;
}

int32_t draw_op(const OpThresholds& th, Draws& dr) {
    const float u = unit(dr.next());
    for (int32_t k = 0; k < 4; ++k)
        if (u < th.t[k]) return k;
    return GP_GENOP_REPRODUCTION;
}

gp_status check_evolve(const gp_evolve_params* e, const char* who) {
    if (!e) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": params is NULL");
    const float ps[5] = {e->p_crossover, e->p_subtree, e->p_hoist, e->p_point, e->p_point_replace};
    for (float v : ps)
        if (!(v >= 0.0f && v <= 1.0f))
            return fail(GP_ERR_INVALID_ARG, std::string(who) + ": probabilities must lie in [0, 1]");
    if (!(thresholds(*e).t[3] <= 1.0f))
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": operation probabilities sum above 1");
    if (e->max_len < 1) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": max_len must be >= 1");
    return GP_OK;
}

}  // namespace
}  // namespace gp

using namespace gp;

extern "C" {

const char* gp_last_error(void) { return g_last_error.c_str(); }

const char* gp_version(void) { return "gp-mi355x 0.1 (gfx950)"; }

int gp_metric_larger_is_better(gp_metric metric) {
    switch (metric) {
    case GP_METRIC_MAE: case GP_METRIC_MSE: case GP_METRIC_RMSE: case GP_METRIC_LOGLOSS:
    case GP_METRIC_USER_0: case GP_METRIC_USER_1: case GP_METRIC_USER_2: case GP_METRIC_USER_3:
        return 0;
    case GP_METRIC_PEARSON: case GP_METRIC_SPEARMAN:
        return 1;
    default:
        return -1;
    }
}

gp_status gp_register_function(uint32_t op, const uint32_t* def, int32_t def_len, const float* consts,
                               int32_t n_consts) {
    if (!is_user_op(op))
        return fail(GP_ERR_INVALID_ARG, "gp_register_function: op must be a user opcode (24..31)");
    const int ar = arity(op);
    const int u = static_cast<int>(op - GP_OP_USER1);
    if (def_len == 0) {
        std::lock_guard<std::mutex> lk(g_user_mu);
        g_user.len[u] = 0;
        g_user_mask.fetch_and(~(1u << op));
        return ok();
    }
    if (!def || def_len < 0 || def_len > GP_USER_MAX_NODES)
        return fail(GP_ERR_INVALID_ARG, "gp_register_function: need 1 <= def_len <= 32 and a definition");
    if (n_consts < 0 || n_consts > GP_USER_MAX_CONSTS || (n_consts > 0 && !consts))
        return fail(GP_ERR_INVALID_ARG, "gp_register_function: need 0 <= n_consts <= 16 and the constants");
    // a valid prefix list over built-in functions, its arguments and its
    // constants, on a stack of at most GP_USER_MAX_STACK values
    int h = 0;
    for (int32_t i = def_len - 1; i >= 0; --i) {
        const uint32_t w = def[i], dop = GP_NODE_OP(w), arg = GP_NODE_ARG(w);
        const int a = dop < GP_OP_COUNT ? arity(dop) : -1;
        if (a < 0)
            return fail(GP_ERR_INVALID_PROGRAM, "gp_register_function: a definition uses built-in functions only");
        if (dop == GP_OP_VAR && arg >= static_cast<uint32_t>(ar))
            return fail(GP_ERR_INVALID_PROGRAM, "gp_register_function: argument index above the arity");
        if (dop == GP_OP_CONST && arg >= static_cast<uint32_t>(n_consts))
            return fail(GP_ERR_INVALID_PROGRAM, "gp_register_function: constant index out of range");
        if (h < a) return fail(GP_ERR_INVALID_PROGRAM, "gp_register_function: a function lacks operands");
        h += 1 - a;
        if (h > GP_USER_MAX_STACK)
            return fail(GP_ERR_STACK_OVERFLOW, "gp_register_function: the definition needs more than 6 stack values");
    }
    if (h != 1) return fail(GP_ERR_INVALID_PROGRAM, "gp_register_function: the definition leaves more than one value");
    std::lock_guard<std::mutex> lk(g_user_mu);
    g_user.len[u] = def_len;
    for (int32_t i = 0; i < GP_USER_MAX_NODES; ++i) g_user.nodes[u][i] = i < def_len ? def[i] : 0u;
    for (int32_t i = 0; i < GP_USER_MAX_CONSTS; ++i) g_user.consts[u][i] = i < n_consts ? consts[i] : 0.0f;
    g_user_mask.fetch_or(1u << op);
    return ok();
}

int gp_function_defined(uint32_t op) { return is_user_op(op) && ((user_defined_mask() >> op) & 1u) ? 1 : 0; }

gp_status gp_build_population(const gp_init_params* prm, uint32_t* nodes, int64_t nodes_cap,
                              int64_t* prog_off, float* consts, int64_t consts_cap,
                              int64_t* const_off, int32_t* len, int64_t* total_nodes,
                              int64_t* total_consts) {
    if (!prm) return fail(GP_ERR_INVALID_ARG, "gp_build_population: params is NULL");
    const gp_init_params& p = *prm;
    gp_status rc = check_init(p, "gp_build_population");
    if (rc != GP_OK) return rc;
    if (nodes && (!prog_off || !const_off || !len || (consts_cap > 0 && !consts)))
        return fail(GP_ERR_INVALID_ARG, "gp_build_population: output arrays must be given with nodes");

    Gen gen(p);
    int64_t n_nodes = 0, n_consts = 0;
    bool short_buf = false;
    for (int32_t prog = 0; prog < p.n_programs; ++prog) {
        Draws dr(p.seed, static_cast<uint32_t>(prog), 0u, kStreamInit);
        gen.program(dr);
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
    const uint32_t user_mask = user_defined_mask();
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
            if (is_user_op(op) && !((user_mask >> op) & 1u))
                return bad(GP_ERR_INVALID_PROGRAM, "user function not defined");
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

gp_status gp_plan_generation(const gp_evolve_params* params, int32_t n_offspring, uint64_t generation,
                             int32_t* ops, int32_t* first_tournament, int32_t* n_tournaments) {
    gp_status rc = check_evolve(params, "gp_plan_generation");
    if (rc != GP_OK) return rc;
    if (n_offspring < 0 || generation > 0xffffffffull || !n_tournaments || (n_offspring > 0 && (!ops || !first_tournament)))
        return fail(GP_ERR_INVALID_ARG, "gp_plan_generation: bad arguments");
    const OpThresholds th = thresholds(*params);
    int64_t t = 0;
    for (int32_t i = 0; i < n_offspring; ++i) {
        Draws dr(params->seed, static_cast<uint32_t>(i), static_cast<uint32_t>(generation), kStreamMutation);
        ops[i] = draw_op(th, dr);
        first_tournament[i] = static_cast<int32_t>(t);
        t += ops[i] == GP_GENOP_CROSSOVER ? 2 : 1;
        if (t > 0x7fffffff) return fail(GP_ERR_INVALID_ARG, "gp_plan_generation: too many tournaments");
    }
    *n_tournaments = static_cast<int32_t>(t);
    return ok();
}

gp_status gp_mutate(const gp_evolve_params* params, const gp_init_params* init, const uint32_t* nodes,
                    const int64_t* prog_off, const float* consts, const int64_t* const_off, int32_t n_parents,
                    const int32_t* ops, const int32_t* first_tournament, const int32_t* winners, int32_t n_winners,
                    int32_t n_offspring, uint64_t generation, uint32_t* out_nodes, int64_t nodes_cap,
                    int64_t* out_prog_off, float* out_consts, int64_t consts_cap, int64_t* out_const_off,
                    int32_t* out_len, int64_t* total_nodes, int64_t* total_consts) {
    gp_status rc = check_evolve(params, "gp_mutate");
    if (rc != GP_OK) return rc;
    if (!init) return fail(GP_ERR_INVALID_ARG, "gp_mutate: init params are NULL");
    rc = check_init(*init, "gp_mutate");
    if (rc != GP_OK) return rc;
    if (n_parents < 1 || n_offspring < 0 || n_winners < 0 || generation > 0xffffffffull || !total_nodes ||
        !total_consts || !out_prog_off || !out_const_off || (n_offspring > 0 && (!ops || !first_tournament || !out_len)) ||
        (n_winners > 0 && !winners))
        return fail(GP_ERR_INVALID_ARG, "gp_mutate: bad arguments");
    // the parents must be valid programs over init->n_features
    rc = gp_validate_population(nodes, prog_off, const_off, n_parents, init->n_features, nullptr, nullptr);
    if (rc != GP_OK) return rc;
    if (const_off[n_parents] > 0 && !consts) return fail(GP_ERR_INVALID_ARG, "gp_mutate: consts is NULL");
    for (int32_t i = 0; i < n_offspring; ++i) {
        const int32_t need = ops[i] == GP_GENOP_CROSSOVER ? 2 : 1;
        if (ops[i] < 0 || ops[i] > GP_GENOP_REPRODUCTION || first_tournament[i] < 0 ||
            static_cast<int64_t>(first_tournament[i]) + need > n_winners)
            return fail(GP_ERR_INVALID_ARG, "gp_mutate: operation or tournament index out of range at offspring " +
                                                std::to_string(i));
        for (int32_t k = 0; k < need; ++k) {
            const int32_t wv = winners[first_tournament[i] + k];
            if (wv < 0 || wv >= n_parents)
                return fail(GP_ERR_INVALID_ARG, "gp_mutate: winner index out of range at offspring " + std::to_string(i));
        }
    }
    const Gen gen(*init);
    Gen donor_gen(*init);
    int64_t n_nodes = 0, n_consts = 0;
    bool short_buf = false;
    for (int32_t i = 0; i < n_offspring; ++i) {
        Draws dr(params->seed, static_cast<uint32_t>(i), static_cast<uint32_t>(generation), kStreamMutation);
        (void)dr.next();   // the operation draw (gp_plan_generation)
        const Prog parent = load_prog(nodes, prog_off, consts, const_off, winners[first_tournament[i]]);
        Prog child;
        switch (ops[i]) {
        case GP_GENOP_CROSSOVER: {
            const Prog donor = load_prog(nodes, prog_off, consts, const_off, winners[first_tournament[i] + 1]);
            child = crossover(parent, donor, dr, params->max_len);
            break;
        }
        case GP_GENOP_SUBTREE: {
            Draws ddr(params->seed, static_cast<uint32_t>(i), static_cast<uint32_t>(generation), kStreamDonor);
            donor_gen.program(ddr);
            child = crossover(parent, from_gen(donor_gen), dr, params->max_len);
            break;
        }
        case GP_GENOP_HOIST: child = hoist(parent, dr); break;
        case GP_GENOP_POINT: child = point(parent, gen, params->p_point_replace, dr); break;
        default: child = parent; break;
        }
        out_prog_off[i] = n_nodes;
        out_const_off[i] = n_consts;
        out_len[i] = static_cast<int32_t>(child.w.size());
        int64_t nc = 0;
        for (uint32_t w : child.w) nc += GP_NODE_OP(w) == GP_OP_CONST;
        if (n_nodes + static_cast<int64_t>(child.w.size()) > nodes_cap || n_consts + nc > consts_cap || !out_nodes ||
            (nc > 0 && !out_consts)) {
            short_buf = true;
        } else {
            uint32_t slot = 0;
            for (size_t j = 0; j < child.w.size(); ++j) {
                uint32_t w = child.w[j];
                if (GP_NODE_OP(w) == GP_OP_CONST) {
                    out_consts[n_consts + slot] = child.val[j];
                    w = GP_NODE(GP_OP_CONST, slot++);
                }
                out_nodes[n_nodes + static_cast<int64_t>(j)] = w;
            }
        }
        n_nodes += static_cast<int64_t>(child.w.size());
        n_consts += nc;
    }
    out_prog_off[n_offspring] = n_nodes;
    out_const_off[n_offspring] = n_consts;
    *total_nodes = n_nodes;
    *total_consts = n_consts;
    if (short_buf) return fail(GP_ERR_BUFFER_TOO_SMALL, "gp_mutate: nodes_cap or consts_cap too small");
    return ok();
}

}  // extern "C"
