// gp_mutate.hip -- the genetic operations of a generation on the device, one
// lane per offspring, with the draws, choices and output layout of the host
// gp_mutate (so the two agree bit for bit).
//
// Sec. II-A lists the operations (crossover, subtree, hoist and point
// mutation, reproduction) and Sec. III-C2 gives hoisted crossover; the paper
// applies them on the CPU, which costs a host round trip per generation.
// Here a generation's offspring come from a short pipeline on one stream:
//   k_plan          the operation of every offspring (draw 0 of stream 2)
//                   and where its tournaments start (a block scan);
//   k_donor<0>      length and constant count of every subtree-mutation
//                   donor (the initialisation method on stream 3);
//   k_scan2         donor offsets;
//   k_donor<1>      the donors, written;
//   k_child<0>      every offspring's splice, length and constant count;
//   k_scan2         offspring offsets (nodes and constants), totals;
//   k_child<1>      the offspring, constants renumbered in prefix order.
// Every launch has a fixed shape, so a generation can be captured in a graph.
// The generation number may be read from device memory, so one captured
// graph serves every generation.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kMutBlock = 64;     // one wave per block
constexpr int kScanBlock = 1024;
constexpr int kPendMax = 32;      // pending depths of a tree walk (<= max depth + 1)

// Counter-based draws of one offspring: words of Philox4x32-10 with counter
// (block, item, generation, tag), consumed in order (the host's Draws).
struct DevDraws {
    uint64_t seed;
    uint32_t item, gen, tag, n;
    uint32_t w0, w1, w2, w3;
    __device__ DevDraws(uint64_t s, uint32_t i, uint32_t g, uint32_t t)
        : seed(s), item(i), gen(g), tag(t), n(0), w0(0), w1(0), w2(0), w3(0) {}
    __device__ uint32_t next() {
        const uint32_t k = n & 3u;
        if (k == 0u) {
            const Philox4 b = philox4x32_10(n >> 2, item, gen, tag, seed);
            w0 = b.v[0];
            w1 = b.v[1];
            w2 = b.v[2];
            w3 = b.v[3];
        }
        ++n;
        return k == 0u ? w0 : (k == 1u ? w1 : (k == 2u ? w2 : w3));
    }
};

// The initialisation settings the generators and point mutation read, with
// the enabled functions in opcode order (all, unary, binary).
struct InitDev {
    int32_t n_features, method, min_depth, max_depth, min_len, max_len, max_consts;
    int32_t consts_enabled;
    float const_lo, const_hi;
    int32_t n_all, n_un, n_bin;
    uint8_t all[GP_OP_LIMIT], un[GP_OP_LIMIT], bin[GP_OP_LIMIT];
};

struct EvolveDev {
    float th[4];          // float32 running sums of the operation probabilities
    float p_point_replace;
    int32_t max_len;
    uint64_t seed;
};

// A read-only population: program p is nodes[off[p] .. off[p+1]), constants
// consts[coff[p] ..).
struct ProgSet {
    const uint32_t* nodes;
    const int64_t* off;
    const float* consts;
    const int64_t* coff;
    int32_t n;
};

__device__ __forceinline__ uint32_t resolve_gen(uint32_t gen, const uint32_t* d_gen) {
    return d_gen ? *d_gen : gen;
}

// The function tables, copied to LDS once per block so that a drawn index
// reads them without local-memory indexing.
struct FnLds {
    uint8_t all[GP_OP_LIMIT], un[GP_OP_LIMIT], bin[GP_OP_LIMIT];
};

__device__ __forceinline__ void load_fns(FnLds& f, const InitDev& in) {
    for (int i = threadIdx.x; i < GP_OP_LIMIT; i += blockDim.x) {
        f.all[i] = in.all[i];
        f.un[i] = in.un[i];
        f.bin[i] = in.bin[i];
    }
    __syncthreads();
}

__device__ __forceinline__ bool const_available(const InitDev& in, int used) {
    return in.consts_enabled && (in.max_consts <= 0 || used < in.max_consts);
}

__device__ __forceinline__ float draw_const(const InitDev& in, DevDraws& dr) {
    const float u = unit(dr.next());
    const float span = in.const_hi - in.const_lo;
    const float scaled = span * u;
    return in.const_lo + scaled;
}

// ---------------------------------------------------------------------------
// Program generation by the initialisation method (Sec. II-A), as the host's
// Gen::program.  WRITE = false only counts nodes and constants; WRITE = true
// writes the nodes to nodes[0..) and the constants, numbered in prefix
// order, to consts[0..); the exact-length walk needs the constant count of
// the counting pass to number right to left.
// ---------------------------------------------------------------------------
template <bool WRITE>
__device__ void gen_tree(const InitDev& in, const FnLds& f, DevDraws& dr, int target, bool full, int8_t* pend,
                         uint32_t* nodes, float* consts, int64_t* n_nodes, int64_t* n_consts) {
    int np = 1;
    pend[0] = 0;
    int used = 0;
    int64_t pos = 0;
    const int nf = in.n_features;
    while (np > 0) {
        const int depth = pend[--np];
        const int n_term = nf + (const_available(in, used) ? 1 : 0);
        int pick;
        bool func;
        if (depth == target) {
            func = false;
            pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(n_term)));
        } else if (depth == 0 || full) {
            func = true;
            pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(in.n_all)));
        } else {
            const int nall = in.n_all + n_term;
            pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(nall)));
            func = pick < in.n_all;
            if (!func) pick -= in.n_all;
        }
        if (func) {
            const uint32_t op = f.all[pick];
            if (WRITE) nodes[pos] = GP_NODE(op, 0);
            const int a = arity(op);
            for (int k = 0; k < a && np < kPendMax; ++k) pend[np++] = static_cast<int8_t>(depth + 1);
        } else if (pick < nf) {
            if (WRITE) nodes[pos] = GP_NODE(GP_OP_VAR, pick);
        } else {
            const float c = draw_const(in, dr);
            if (WRITE) {
                nodes[pos] = GP_NODE(GP_OP_CONST, used);
                consts[used] = c;
            }
            ++used;
        }
        ++pos;
    }
    *n_nodes = pos;
    *n_consts = used;
}

template <bool WRITE>
__device__ void gen_exact(const InitDev& in, const FnLds& f, DevDraws& dr, int64_t nc_total, uint32_t* nodes,
                          float* consts, int64_t* n_nodes, int64_t* n_consts) {
    uint32_t L = static_cast<uint32_t>(in.min_len) +
                 below(dr.next(), static_cast<uint32_t>(in.max_len - in.min_len + 1));
    const bool no_unary = in.n_un == 0;
    if (no_unary && (L % 2u) == 0u)
        L = (L - 1 >= static_cast<uint32_t>(in.min_len) && L > 1) ? L - 1 : L + 1;
    int h = 0;
    int64_t nc = 0;
    const int nf = in.n_features;
    for (int i = static_cast<int>(L) - 1; i >= 0; --i) {
        const int n_term = nf + (const_available(in, static_cast<int>(nc)) ? 1 : 0);
        bool t_ok = h + 1 <= GP_MAX_STACK && h <= i;
        const bool u_ok = !no_unary && h >= 1 && h - 1 <= i;
        bool b_ok = in.n_bin > 0 && h >= 2 && h - 2 <= i;
        if (no_unary) {
            if (t_ok && ((h + i) & 1)) t_ok = false;
            if (b_ok && ((h - 2 + i) & 1)) b_ok = false;
        }
        const int nt = t_ok ? n_term : 0;
        const int nu = u_ok ? in.n_un : 0;
        const int nb = b_ok ? in.n_bin : 0;
        int pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(nt + nu + nb)));
        if (pick < nt) {
            if (pick < nf) {
                if (WRITE) nodes[i] = GP_NODE(GP_OP_VAR, pick);
            } else {
                const float c = draw_const(in, dr);
                if (WRITE) {
                    // generated right to left, numbered left to right
                    const int64_t slot = nc_total - 1 - nc;
                    nodes[i] = GP_NODE(GP_OP_CONST, static_cast<uint32_t>(slot));
                    consts[slot] = c;
                }
                ++nc;
            }
            ++h;
        } else if ((pick -= nt) < nu) {
            if (WRITE) nodes[i] = GP_NODE(f.un[pick], 0);
        } else {
            if (WRITE) nodes[i] = GP_NODE(f.bin[pick - nu], 0);
            --h;
        }
    }
    *n_nodes = L;
    *n_consts = nc;
}

template <bool WRITE>
__device__ void gen_program(const InitDev& in, const FnLds& f, DevDraws& dr, int8_t* pend, int64_t nc_total,
                            uint32_t* nodes, float* consts, int64_t* n_nodes, int64_t* n_consts) {
    if (in.method == GP_INIT_EXACT_LEN) {
        gen_exact<WRITE>(in, f, dr, nc_total, nodes, consts, n_nodes, n_consts);
        return;
    }
    bool full;
    if (in.method == GP_INIT_RHH) full = !(unit(dr.next()) < 0.5f);
    else full = in.method == GP_INIT_FULL;
    const int depth = in.min_depth +
                      static_cast<int>(below(dr.next(), static_cast<uint32_t>(in.max_depth - in.min_depth + 1)));
    gen_tree<WRITE>(in, f, dr, depth, full, pend, nodes, consts, n_nodes, n_consts);
}

// ---------------------------------------------------------------------------
// k_plan: one block.  ops[i] from draw 0 of (seed, i, generation, stream 2);
// first[i] = sum over j < i of (2 for crossover, else 1); *n_tournaments =
// the total.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kScanBlock) void k_plan(EvolveDev ev, int32_t n, uint32_t gen, const uint32_t* d_gen,
                                                     int32_t* __restrict__ ops, int32_t* __restrict__ first,
                                                     int32_t* __restrict__ n_tournaments) {
    __shared__ int32_t wsum[kScanBlock / 64];
    __shared__ int32_t carry_s;
    const uint32_t g = resolve_gen(gen, d_gen);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int32_t base = 0; base < n; base += kScanBlock) {
        const int32_t i = base + static_cast<int32_t>(threadIdx.x);
        int32_t t = 0;
        if (i < n) {
            DevDraws dr(ev.seed, static_cast<uint32_t>(i), g, kStreamMutation);
            const float u = unit(dr.next());
            int32_t op = GP_GENOP_REPRODUCTION;
            for (int k = 3; k >= 0; --k)
                if (u < ev.th[k]) op = k;
            ops[i] = op;
            t = op == GP_GENOP_CROSSOVER ? 2 : 1;
        }
        // inclusive scan within the wave, then across the block's waves
        int32_t v = t;
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t o = __shfl_up(v, d, 64);
            if (lane >= d) v += o;
        }
        if (lane == 63) wsum[wid] = v;
        __syncthreads();
        int32_t before = carry_s;
        for (int k = 0; k < wid; ++k) before += wsum[k];
        if (i < n) first[i] = before + v - t;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) carry_s = before + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_tournaments = carry_s;
}

// ---------------------------------------------------------------------------
// k_scan2: one block.  out_a[i] = sum of a[j < i] (i = 0..n), likewise b;
// info[0], info[1] = the totals; a total above its capacity sets info[2].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kScanBlock) void k_scan2(const int64_t* __restrict__ a, const int64_t* __restrict__ b,
                                                      int32_t n, int64_t* __restrict__ out_a,
                                                      int64_t* __restrict__ out_b, int64_t cap_a, int64_t cap_b,
                                                      int64_t* __restrict__ info) {
    __shared__ int64_t wa[kScanBlock / 64], wb[kScanBlock / 64];
    __shared__ int64_t ca, cb;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        ca = 0;
        cb = 0;
    }
    __syncthreads();
    for (int32_t base = 0; base < n; base += kScanBlock) {
        const int32_t i = base + static_cast<int32_t>(threadIdx.x);
        const int64_t ta = i < n ? a[i] : 0, tb = i < n ? b[i] : 0;
        int64_t va = ta, vb = tb;
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t oa = __shfl_up(va, d, 64);
            const int64_t ob = __shfl_up(vb, d, 64);
            if (lane >= d) {
                va += oa;
                vb += ob;
            }
        }
        if (lane == 63) {
            wa[wid] = va;
            wb[wid] = vb;
        }
        __syncthreads();
        int64_t pa = ca, pb = cb;
        for (int k = 0; k < wid; ++k) {
            pa += wa[k];
            pb += wb[k];
        }
        if (i < n) {
            out_a[i] = pa + va - ta;
            out_b[i] = pb + vb - tb;
        }
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) {
            ca = pa + va;
            cb = pb + vb;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out_a[n] = ca;
        out_b[n] = cb;
        if (info) {
            info[0] = ca;
            info[1] = cb;
            if (ca > cap_a || cb > cap_b) info[2] |= 1;
        }
    }
}

// Clears the status word before a pipeline (a fill kernel, not a memset, so
// that a captured graph replays it).
__global__ void k_mut_reset(int64_t* __restrict__ info) {
    if (threadIdx.x < 4) info[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// k_donor<WRITE>: one lane per offspring; only subtree-mutation offspring
// have a donor.
// ---------------------------------------------------------------------------
template <bool WRITE>
__global__ __launch_bounds__(kMutBlock) void k_donor(InitDev in, EvolveDev ev, int32_t n, uint32_t gen,
                                                     const uint32_t* d_gen, const int32_t* __restrict__ ops,
                                                     int64_t* __restrict__ dlen, int64_t* __restrict__ dnc,
                                                     const int64_t* __restrict__ doff,
                                                     const int64_t* __restrict__ dcoff, uint32_t* __restrict__ dnodes,
                                                     float* __restrict__ dconsts, int64_t donor_cap,
                                                     int64_t* __restrict__ info) {
    __shared__ FnLds f;
    __shared__ int8_t pend[kMutBlock][kPendMax];
    load_fns(f, in);
    const int32_t i = blockIdx.x * kMutBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t op = ops[i];
    if (op != GP_GENOP_SUBTREE) {
        if (!WRITE) {
            dlen[i] = 0;
            dnc[i] = 0;
        }
        return;
    }
    const uint32_t g = resolve_gen(gen, d_gen);
    DevDraws dr(ev.seed, static_cast<uint32_t>(i), g, kStreamDonor);
    int64_t nn = 0, nc = 0;
    if (!WRITE) {
        gen_program<false>(in, f, dr, pend[threadIdx.x], 0, nullptr, nullptr, &nn, &nc);
        dlen[i] = nn;
        dnc[i] = nc;
        return;
    }
    // the donors must fit the library's buffer (their bound is exact, so
    // this does not happen for valid settings); otherwise nothing is written
    // and k_child treats every subtree-mutation offspring as invalid
    if (doff[n] > donor_cap || dcoff[n] > donor_cap) {
        atomicOr(reinterpret_cast<unsigned long long*>(info + 2), 4ull);
        return;
    }
    gen_program<true>(in, f, dr, pend[threadIdx.x], dlen[i] > 0 ? dnc[i] : 0, dnodes + doff[i], dconsts + dcoff[i], &nn,
                      &nc);
}

// ---------------------------------------------------------------------------
// Splice arithmetic on read-only programs.
// ---------------------------------------------------------------------------
// One past the last node of the subtree rooted at s (bounded by len).
__device__ __forceinline__ int64_t subtree_end(const uint32_t* w, int64_t len, int64_t s) {
    int open = 1;
    int64_t i = s;
    while (open > 0 && i < len) {
        open += arity(GP_NODE_OP(w[i])) - 1;
        ++i;
    }
    return i;
}

// Peak height of the right-to-left scan of parent[0:s) + donor[ds:de) + parent[e:L).
__device__ int splice_peak(const uint32_t* pw, int64_t L, int64_t s, int64_t e, const uint32_t* dw, int64_t ds,
                           int64_t de) {
    int h = 0, hmax = 0;
    for (int64_t i = L - 1; i >= e; --i) {
        h += 1 - arity(GP_NODE_OP(pw[i]));
        hmax = max(hmax, h);
    }
    for (int64_t i = de - 1; i >= ds; --i) {
        h += 1 - arity(GP_NODE_OP(dw[i]));
        hmax = max(hmax, h);
    }
    for (int64_t i = s - 1; i >= 0; --i) {
        h += 1 - arity(GP_NODE_OP(pw[i]));
        hmax = max(hmax, h);
    }
    return hmax;
}

__device__ __forceinline__ int64_t count_consts(const uint32_t* w, int64_t a, int64_t b) {
    int64_t c = 0;
    for (int64_t i = a; i < b; ++i) c += GP_NODE_OP(w[i]) == GP_OP_CONST;
    return c;
}

// Copies w[a:b) to out, constants renumbered from *slot (values from cv by
// their old slot).
__device__ __forceinline__ void copy_seg(const uint32_t* w, const float* cv, int64_t a, int64_t b, uint32_t* out,
                                         float* oc, int64_t* pos, uint32_t* slot) {
    for (int64_t i = a; i < b; ++i) {
        uint32_t x = w[i];
        if (GP_NODE_OP(x) == GP_OP_CONST) {
            oc[*slot] = cv[GP_NODE_ARG(x)];
            x = GP_NODE(GP_OP_CONST, *slot);
            ++*slot;
        }
        out[(*pos)++] = x;
    }
}

// ---------------------------------------------------------------------------
// k_child<WRITE>: one lane per offspring.  WRITE = false draws the splice
// (crossover / subtree: parent cut (s, e) and donor subtree (ds, de) after
// hoisting; hoist: (s, e) and (s2, e2)), stores it in plan[i] and the child's
// length and constant count; WRITE = true writes the child.  Point mutation
// re-draws in both passes.  An index out of range (operation, tournament,
// winner) sets info[2] bit 2 and yields the one-node program x0.
// ---------------------------------------------------------------------------
template <bool WRITE>
__global__ __launch_bounds__(kMutBlock) void k_child(
    InitDev in, EvolveDev ev, ProgSet par, ProgSet don, int32_t n, uint32_t gen, const uint32_t* d_gen,
    const int32_t* __restrict__ ops, const int32_t* __restrict__ first, const int32_t* __restrict__ winners,
    int32_t n_winners, int4* __restrict__ plan, int64_t* __restrict__ clen, int64_t* __restrict__ cnc,
    const int64_t* __restrict__ coff, const int64_t* __restrict__ ccoff, uint32_t* __restrict__ out_nodes,
    float* __restrict__ out_consts, int32_t* __restrict__ out_len, int64_t nodes_cap, int64_t consts_cap,
    int64_t donor_cap, int64_t* __restrict__ info) {
    __shared__ FnLds f;
    load_fns(f, in);
    const int32_t i = blockIdx.x * kMutBlock + threadIdx.x;
    if (i >= n) return;
    if (WRITE) {
        if (coff[n] > nodes_cap || ccoff[n] > consts_cap) return;   // flagged by k_scan2
    }
    const int32_t op = ops[i];
    const int32_t need = op == GP_GENOP_CROSSOVER ? 2 : 1;
    const int32_t t0 = first[i];
    bool bad = op < 0 || op > GP_GENOP_REPRODUCTION || t0 < 0 || static_cast<int64_t>(t0) + need > n_winners;
    if (op == GP_GENOP_SUBTREE && (don.off[don.n] > donor_cap || don.coff[don.n] > donor_cap)) bad = true;
    int32_t pa = 0, pb = 0;
    if (!bad) {
        pa = winners[t0];
        pb = need == 2 ? winners[t0 + 1] : 0;
        bad = pa < 0 || pa >= par.n || pb < 0 || pb >= par.n;
    }
    if (bad) {
        if (!WRITE) {
            atomicOr(reinterpret_cast<unsigned long long*>(info + 2), 2ull);
            clen[i] = 1;
            cnc[i] = 0;
        } else {
            out_nodes[coff[i]] = GP_NODE(GP_OP_VAR, 0);
            out_len[i] = 1;
        }
        return;
    }
    const uint32_t g = resolve_gen(gen, d_gen);
    DevDraws dr(ev.seed, static_cast<uint32_t>(i), g, kStreamMutation);
    (void)dr.next();   // the operation draw
    const uint32_t* pw = par.nodes + par.off[pa];
    const float* pc = par.consts + par.coff[pa];
    const int64_t L = par.off[pa + 1] - par.off[pa];
    uint32_t* on = out_nodes + (WRITE ? coff[i] : 0);
    float* oc = out_consts + (WRITE ? ccoff[i] : 0);
    int64_t pos = 0;
    uint32_t slot = 0;

    if (op == GP_GENOP_CROSSOVER || op == GP_GENOP_SUBTREE) {
        const uint32_t* dw;
        const float* dc;
        int64_t DL;
        if (op == GP_GENOP_CROSSOVER) {
            dw = par.nodes + par.off[pb];
            dc = par.consts + par.coff[pb];
            DL = par.off[pb + 1] - par.off[pb];
        } else {
            dw = don.nodes + don.off[i];
            dc = don.consts + don.coff[i];
            DL = don.off[i + 1] - don.off[i];
        }
        int64_t s, e, ds, de;
        if (!WRITE) {
            s = below(dr.next(), static_cast<uint32_t>(L));
            e = subtree_end(pw, L, s);
            ds = below(dr.next(), static_cast<uint32_t>(DL));
            de = subtree_end(dw, DL, ds);
            for (;;) {
                const int64_t clen_try = L - (e - s) + (de - ds);
                const bool fits = splice_peak(pw, L, s, e, dw, ds, de) <= GP_MAX_STACK && clen_try <= ev.max_len;
                if (fits || de - ds == 1) break;
                ds = ds + 1 + below(dr.next(), static_cast<uint32_t>(de - ds - 1));
                de = subtree_end(dw, DL, ds);
            }
            plan[i] = make_int4(static_cast<int>(s), static_cast<int>(e), static_cast<int>(ds), static_cast<int>(de));
            clen[i] = L - (e - s) + (de - ds);
            cnc[i] = count_consts(pw, 0, s) + count_consts(dw, ds, de) + count_consts(pw, e, L);
        } else {
            const int4 q = plan[i];
            s = q.x;
            e = q.y;
            ds = q.z;
            de = q.w;
            copy_seg(pw, pc, 0, s, on, oc, &pos, &slot);
            copy_seg(dw, dc, ds, de, on, oc, &pos, &slot);
            copy_seg(pw, pc, e, L, on, oc, &pos, &slot);
            out_len[i] = static_cast<int32_t>(pos);
        }
        return;
    }
    if (op == GP_GENOP_HOIST) {
        if (!WRITE) {
            const int64_t s = below(dr.next(), static_cast<uint32_t>(L));
            const int64_t e = subtree_end(pw, L, s);
            const int64_t s2 = s + below(dr.next(), static_cast<uint32_t>(e - s));
            const int64_t e2 = subtree_end(pw, L, s2);
            plan[i] = make_int4(static_cast<int>(s), static_cast<int>(e), static_cast<int>(s2), static_cast<int>(e2));
            clen[i] = L - (e - s) + (e2 - s2);
            cnc[i] = count_consts(pw, 0, s) + count_consts(pw, s2, e2) + count_consts(pw, e, L);
        } else {
            const int4 q = plan[i];
            copy_seg(pw, pc, 0, q.x, on, oc, &pos, &slot);
            copy_seg(pw, pc, q.z, q.w, on, oc, &pos, &slot);
            copy_seg(pw, pc, q.y, L, on, oc, &pos, &slot);
            out_len[i] = static_cast<int32_t>(pos);
        }
        return;
    }
    if (op == GP_GENOP_POINT) {
        int n_const = static_cast<int>(count_consts(pw, 0, L));
        const int nf = in.n_features;
        for (int64_t j = 0; j < L; ++j) {
            uint32_t x = pw[j];
            float v = 0.0f;
            const uint32_t xop = GP_NODE_OP(x);
            if (xop == GP_OP_CONST) v = pc[GP_NODE_ARG(x)];
            if (unit(dr.next()) < ev.p_point_replace) {
                const int ar = arity(xop);
                if (ar > 0) {
                    const int ns = ar == 1 ? in.n_un : in.n_bin;
                    if (ns > 0) {
                        const uint32_t k = below(dr.next(), static_cast<uint32_t>(ns));
                        x = GP_NODE(ar == 1 ? f.un[k] : f.bin[k], 0);
                    }
                } else {
                    const int others = n_const - (xop == GP_OP_CONST ? 1 : 0);
                    const int n_term = nf + (const_available(in, others) ? 1 : 0);
                    const int pick = static_cast<int>(below(dr.next(), static_cast<uint32_t>(n_term)));
                    if (pick < nf) {
                        x = GP_NODE(GP_OP_VAR, pick);
                        n_const = others;
                    } else {
                        x = GP_NODE(GP_OP_CONST, 0);
                        v = draw_const(in, dr);
                        n_const = others + 1;
                    }
                }
            }
            if (WRITE) {
                if (GP_NODE_OP(x) == GP_OP_CONST) {
                    oc[slot] = v;
                    x = GP_NODE(GP_OP_CONST, slot);
                    ++slot;
                }
                on[pos] = x;
            }
            ++pos;
        }
        if (!WRITE) {
            clen[i] = L;
            cnc[i] = n_const;
        } else {
            out_len[i] = static_cast<int32_t>(pos);
        }
        return;
    }
    // reproduction
    if (!WRITE) {
        clen[i] = L;
        cnc[i] = count_consts(pw, 0, L);
    } else {
        copy_seg(pw, pc, 0, L, on, oc, &pos, &slot);
        out_len[i] = static_cast<int32_t>(pos);
    }
}

// Programs longer than the donor capacity cannot come from these settings:
// the largest donor the initialisation method can produce.
int64_t donor_bound(const gp_init_params& in) {
    if (in.method == GP_INIT_EXACT_LEN) return static_cast<int64_t>(in.max_len) + 1;
    bool has_binary = false;
    for (uint32_t op = GP_OP_ADD; op < GP_OP_LIMIT; ++op)
        has_binary |= arity(op) == 2 && ((in.function_mask >> op) & 1u);
    return has_binary ? (int64_t{1} << (in.max_depth + 1)) - 1 : in.max_depth + 1;
}

InitDev to_dev(const gp_init_params& p) {
    InitDev d{};
    d.n_features = p.n_features;
    d.method = p.method;
    d.min_depth = p.min_depth;
    d.max_depth = p.max_depth;
    d.min_len = p.min_len;
    d.max_len = p.max_len;
    d.max_consts = p.max_consts;
    d.consts_enabled = !(p.const_lo > p.const_hi);
    d.const_lo = p.const_lo;
    d.const_hi = p.const_hi;
    for (uint32_t op = GP_OP_ADD; op < GP_OP_LIMIT; ++op) {
        if (!(p.function_mask & (1u << op)) || arity(op) < 1) continue;
        d.all[d.n_all++] = static_cast<uint8_t>(op);
        if (arity(op) == 1) d.un[d.n_un++] = static_cast<uint8_t>(op);
        else d.bin[d.n_bin++] = static_cast<uint8_t>(op);
    }
    return d;
}

EvolveDev to_dev(const gp_evolve_params& e) {
    EvolveDev d{};
    d.th[0] = e.p_crossover;
    d.th[1] = d.th[0] + e.p_subtree;
    d.th[2] = d.th[1] + e.p_hoist;
    d.th[3] = d.th[2] + e.p_point;
    d.p_point_replace = e.p_point_replace;
    d.max_len = e.max_len;
    d.seed = e.seed;
    return d;
}

template <typename T>
gp_status grow_buf(T** p, int64_t* cap, int64_t need) {
    if (*cap >= need && *p) return GP_OK;
    if (*p) {
        GP_HIP(hipDeviceSynchronize());
        GP_HIP(hipFree(*p));
        *p = nullptr;
        *cap = 0;
    }
    const int64_t n = std::max<int64_t>(need, 1);
    if (hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * static_cast<size_t>(n)) != hipSuccess) {
        *p = nullptr;
        return fail(GP_ERR_OUT_OF_MEMORY, "device mutation: hipMalloc failed");
    }
    *cap = n;
    return GP_OK;
}

}  // namespace

gp_status mutate_check(const gp_evolve_params* ev, const gp_init_params* in, int32_t n_offspring, const char* who) {
    if (!ev || !in) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": params are NULL");
    const float ps[5] = {ev->p_crossover, ev->p_subtree, ev->p_hoist, ev->p_point, ev->p_point_replace};
    for (float v : ps)
        if (!(v >= 0.0f && v <= 1.0f))
            return fail(GP_ERR_INVALID_ARG, std::string(who) + ": probabilities must lie in [0, 1]");
    const EvolveDev e = to_dev(*ev);
    if (!(e.th[3] <= 1.0f)) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": operation probabilities sum above 1");
    if (ev->max_len < 1) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": max_len must be >= 1");
    if (n_offspring < 0) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": n_offspring < 0");
    if (in->n_features < 1) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": n_features >= 1");
    if (in->function_mask == 0 || (in->function_mask & ~allowed_function_mask()))
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": function_mask must select functions (bits 2..22, "
                                                           "or 24..31 once defined) only");
    if (in->method == GP_INIT_EXACT_LEN) {
        if (in->min_len < 1 || in->max_len < in->min_len || in->max_len > (1 << 20))
            return fail(GP_ERR_INVALID_ARG, std::string(who) + ": need 1 <= min_len <= max_len <= 2^20");
        if (donor_bound(*in) > 1 && in->max_len > 1) {
            bool has_binary = false;
            for (uint32_t op = GP_OP_ADD; op < GP_OP_LIMIT; ++op)
                has_binary |= arity(op) == 2 && ((in->function_mask >> op) & 1u);
            if (!has_binary)
                return fail(GP_ERR_INVALID_ARG, std::string(who) + ": exact lengths above 1 need a binary function");
        }
    } else if (in->method >= GP_INIT_RHH && in->method <= GP_INIT_GROW) {
        if (in->min_depth < 0 || in->max_depth < in->min_depth || in->max_depth > GP_MAX_STACK - 1)
            return fail(GP_ERR_INVALID_ARG, std::string(who) + ": need 0 <= min_depth <= max_depth <= 19");
    } else {
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": unknown method");
    }
    return GP_OK;
}

gp_status mutate_work_reserve(MutateWork* w, int32_t n_offspring, const gp_init_params& in) {
    const int64_t n1 = static_cast<int64_t>(n_offspring) + 1;
    const int64_t dcap = std::max<int64_t>(donor_bound(in) * std::max<int32_t>(n_offspring, 1), 1);
    if (dcap > (int64_t{1} << 25))
        return fail(GP_ERR_INVALID_ARG, "device mutation: donors of these initialisation settings could need more "
                                        "than 2^25 nodes; lower max_depth / max_len or mutate on the host");
    gp_status rc;
    if ((rc = grow_buf(&w->dlen, &w->dlen_cap, n1)) != GP_OK) return rc;
    if ((rc = grow_buf(&w->dnc, &w->dnc_cap, n1)) != GP_OK) return rc;
    if ((rc = grow_buf(&w->doff, &w->doff_cap, n1)) != GP_OK) return rc;
    if ((rc = grow_buf(&w->dcoff, &w->dcoff_cap, n1)) != GP_OK) return rc;
    if ((rc = grow_buf(&w->clen, &w->clen_cap, n1)) != GP_OK) return rc;
    if ((rc = grow_buf(&w->cnc, &w->cnc_cap, n1)) != GP_OK) return rc;
    if ((rc = grow_buf(&w->plan, &w->plan_cap, n1)) != GP_OK) return rc;
    if ((rc = grow_buf(&w->dnodes, &w->dnodes_cap, dcap)) != GP_OK) return rc;
    if ((rc = grow_buf(&w->dconsts, &w->dconsts_cap, dcap)) != GP_OK) return rc;
    w->donor_cap = std::min(w->dnodes_cap, w->dconsts_cap);
    return GP_OK;
}

void mutate_work_free(MutateWork* w) {
    for (void* p : {static_cast<void*>(w->dlen), static_cast<void*>(w->dnc), static_cast<void*>(w->doff),
                    static_cast<void*>(w->dcoff), static_cast<void*>(w->clen), static_cast<void*>(w->cnc),
                    static_cast<void*>(w->plan), static_cast<void*>(w->dnodes), static_cast<void*>(w->dconsts)})
        if (p) (void)hipFree(p);
    *w = MutateWork{};
}

gp_status plan_launch(const gp_evolve_params& ev, int32_t n_offspring, uint32_t gen, const uint32_t* d_gen,
                      int32_t* ops, int32_t* first, int32_t* n_tournaments, hipStream_t s) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kScanBlock), 0, s, to_dev(ev), n_offspring, gen, d_gen, ops, first,
                       n_tournaments);
    GP_HIP(hipGetLastError());
    return GP_OK;
}

gp_status mutate_launch(MutateWork& w, const gp_evolve_params& evp, const gp_init_params& inp,
                        const gp_population_dev& par, const int32_t* ops, const int32_t* first, const int32_t* winners,
                        int32_t n_winners, int32_t n_offspring, uint32_t gen, const uint32_t* d_gen,
                        const gp_population_out_dev& out, int64_t* info, hipStream_t s) {
    const InitDev in = to_dev(inp);
    const EvolveDev ev = to_dev(evp);
    const int32_t n = n_offspring;
    hipLaunchKernelGGL(k_mut_reset, dim3(1), dim3(64), 0, s, info);
    GP_HIP(hipGetLastError());
    if (n == 0) {
        hipLaunchKernelGGL(k_scan2, dim3(1), dim3(kScanBlock), 0, s, w.clen, w.cnc, 0, out.prog_off, out.const_off,
                           out.node_capacity, out.const_capacity, info);
        GP_HIP(hipGetLastError());
        return GP_OK;
    }
    const dim3 grid((n + kMutBlock - 1) / kMutBlock), blk(kMutBlock);
    hipLaunchKernelGGL(k_donor<false>, grid, blk, 0, s, in, ev, n, gen, d_gen, ops, w.dlen, w.dnc, w.doff, w.dcoff,
                       w.dnodes, w.dconsts, w.donor_cap, info);
    GP_HIP(hipGetLastError());
    // donor overflow is a library bound, not the caller's capacity: bit 3
    hipLaunchKernelGGL(k_scan2, dim3(1), dim3(kScanBlock), 0, s, w.dlen, w.dnc, n, w.doff, w.dcoff, w.donor_cap,
                       w.donor_cap, static_cast<int64_t*>(nullptr));
    GP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_donor<true>, grid, blk, 0, s, in, ev, n, gen, d_gen, ops, w.dlen, w.dnc, w.doff, w.dcoff,
                       w.dnodes, w.dconsts, w.donor_cap, info);
    GP_HIP(hipGetLastError());
    const ProgSet p{par.nodes, par.prog_off, par.consts, par.const_off, par.n_programs};
    const ProgSet d{w.dnodes, w.doff, w.dconsts, w.dcoff, n};
    hipLaunchKernelGGL(k_child<false>, grid, blk, 0, s, in, ev, p, d, n, gen, d_gen, ops, first, winners, n_winners,
                       w.plan, w.clen, w.cnc, static_cast<const int64_t*>(nullptr),
                       static_cast<const int64_t*>(nullptr), out.nodes, out.consts, out.len, out.node_capacity,
                       out.const_capacity, w.donor_cap, info);
    GP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan2, dim3(1), dim3(kScanBlock), 0, s, w.clen, w.cnc, n, out.prog_off, out.const_off,
                       out.node_capacity, out.const_capacity, info);
    GP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_child<true>, grid, blk, 0, s, in, ev, p, d, n, gen, d_gen, ops, first, winners, n_winners,
                       w.plan, w.clen, w.cnc, out.prog_off, out.const_off, out.nodes, out.consts, out.len,
                       out.node_capacity, out.const_capacity, w.donor_cap, info);
    GP_HIP(hipGetLastError());
    return GP_OK;
}

}  // namespace gp

namespace {
std::mutex g_mut_mu;
std::vector<gp::MutateWork> g_mut_work;   // per device
}  // namespace

extern "C" {

gp_status gp_plan_generation_device(const gp_evolve_params* params, int32_t n_offspring, uint64_t generation,
                                    int32_t* ops, int32_t* first_tournament, int32_t* n_tournaments, void* stream) {
    using namespace gp;
    if (!params) return fail(GP_ERR_INVALID_ARG, "gp_plan_generation_device: params is NULL");
    gp_init_params dummy{};
    dummy.n_features = 1;
    dummy.method = GP_INIT_GROW;
    dummy.function_mask = 1u << GP_OP_ADD;
    gp_status rc = mutate_check(params, &dummy, n_offspring, "gp_plan_generation_device");
    if (rc != GP_OK) return rc;
    if (generation > 0xffffffffull || !n_tournaments || (n_offspring > 0 && (!ops || !first_tournament)))
        return fail(GP_ERR_INVALID_ARG, "gp_plan_generation_device: bad arguments");
    if (static_cast<int64_t>(n_offspring) * 2 > 0x7fffffff)
        return fail(GP_ERR_INVALID_ARG, "gp_plan_generation_device: too many offspring");
    return plan_launch(*params, n_offspring, static_cast<uint32_t>(generation), nullptr, ops, first_tournament,
                       n_tournaments, static_cast<hipStream_t>(stream));
}

gp_status gp_mutate_device(const gp_evolve_params* params, const gp_init_params* init,
                           const gp_population_dev* parents, const int32_t* ops, const int32_t* first_tournament,
                           const int32_t* winners, int32_t n_winners, int32_t n_offspring, uint64_t generation,
                           const gp_population_out_dev* out, int64_t* info, void* stream) {
    using namespace gp;
    gp_status rc = mutate_check(params, init, n_offspring, "gp_mutate_device");
    if (rc != GP_OK) return rc;
    if (!parents || !out || !info || generation > 0xffffffffull || n_winners < 0)
        return fail(GP_ERR_INVALID_ARG, "gp_mutate_device: bad arguments");
    if (parents->n_programs < 1 || !parents->nodes || !parents->prog_off || !parents->const_off ||
        (parents->total_consts > 0 && !parents->consts))
        return fail(GP_ERR_INVALID_ARG, "gp_mutate_device: parents need n_programs >= 1 and their arrays");
    if (!out->prog_off || !out->const_off || out->node_capacity < 0 || out->const_capacity < 0 ||
        (n_offspring > 0 && (!out->len || !ops || !first_tournament || !out->nodes || (n_winners > 0 && !winners))) ||
        (out->const_capacity > 0 && !out->consts))
        return fail(GP_ERR_INVALID_ARG, "gp_mutate_device: output arrays missing");
    std::lock_guard<std::mutex> lk(g_mut_mu);
    int dev = 0;
    GP_HIP(hipGetDevice(&dev));
    if (static_cast<int>(g_mut_work.size()) <= dev) g_mut_work.resize(dev + 1);
    MutateWork& w = g_mut_work[dev];
    rc = mutate_work_reserve(&w, n_offspring, *init);
    if (rc != GP_OK) return rc;
    return mutate_launch(w, *params, *init, *parents, ops, first_tournament, winners, n_winners, n_offspring,
                         static_cast<uint32_t>(generation), nullptr, *out, info, static_cast<hipStream_t>(stream));
}

}  // extern "C"
