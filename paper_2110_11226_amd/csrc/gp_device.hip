// gp_device.hip -- gfx950 kernels and the device entry points of the C ABI.
//
// Hot path (Sec. III-C3 of "Accelerating Genetic Programming using GPUs"):
// every program of the population is evaluated on every dataset row by a
// right-to-left stack scan of its prefix list (Sec. III-A), each row's loss
// against the target is formed in registers, and the losses are summed per
// program.  The paper launches one thread per (program, row) and materialises
// the (rows x programs) prediction matrix before two library reductions; here
//   1. k_compile rewrites each prefix list once per call into its execution
//      order as two-word instructions (the stack-schedule pre-pass): a
//      terminal whose parent is a binary function and which is that
//      function's first operand is fused with it, and a constant's value
//      travels inside its instruction;
//   2. one persistent launch of k_eval walks (row chunk, program) work items
//      taken from an atomic counter; the 64 lanes of a wavefront run the same
//      program on 64 different rows, so every instruction is a wave-uniform
//      (scalar) branch, and each lane carries R rows to spread the scalar
//      dispatch over more vector work; the row loss is formed in registers
//      and only one float64 partial per (program, chunk) leaves the kernel;
//   3. k_finalize merges the partials in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "gp_crmath.h"
#include "gp_internal.h"

using namespace gp;

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;                  // 4 independent wavefronts per block
constexpr int kSpill = GP_MAX_STACK - 1;     // stack entries below the cached top

// ---------------------------------------------------------------------------
// Views passed to kernels by value.
// ---------------------------------------------------------------------------
struct PopView {
    const uint32_t* nodes;
    const int64_t* prog_off;
    const float* consts;
    const int64_t* const_off;
    const int32_t* len;
    int32_t P;
};

struct DataView {
    const float* X;
    int64_t ld;
    int32_t F;
    int64_t N;
    const float* y;
    const float* w;
};

// Compiled programs: program p's instructions are code[prog_off[p] ..
// prog_off[p] + clen[p]) (clen[p] <= len[p]), in execution order.
struct CodeView {
    const uint4* code;     // the adjoint's format (k_compile)
    const int32_t* clen;
    const uint4* ecode;    // the evaluation kernel's format (k_compile_eval):
    const int32_t* eclen;  // program p from ecode[prog_off[p] * ex_mul + p * ex_add]
    int32_t ex_mul;        // instructions per node at most (1, or the longest user definition)
    int32_t ex_add;        // instructions per program added by a user loss
};

// Work decomposition: rows are split into n_chunks chunks of `chunk` rows
// (a multiple of the 64*R rows one wavefront covers per tile).  Work item
// it = chunk_index * P + k covers program order[k] on that chunk; programs are
// ordered longest first so each chunk's long programs start early.
// The work counters: one per XCD queue, 64 bytes apart, in a 1 KiB block
// whose word kFlagWord serves the backward pass's user-function check.
constexpr int kQueues = 8;
constexpr int kQueueStride = 16;
constexpr size_t kCounterBytes = 1024;
constexpr int kFlagWord = 128;

struct Sched {
    int64_t chunk;
    int32_t n_chunks;
    int64_t n_items;
    const int32_t* order;
    uint32_t* counter;
    int32_t batch;     // work items claimed per atomic by the evaluation kernel
    int32_t lds_slots; // stack slots per row in LDS (kEvalLds or kEvalLdsUser)
};

// ---------------------------------------------------------------------------
// Instruction format (word x; word y):
//   bits 0-1  class: kPush (push a terminal), kFold (terminal fused with the
//             binary function whose first operand it is; the current top is
//             the second operand), kBin (binary: top op next-below), kUn
//   bits 2-5  function: binary ADD..DIV, MAX..ATAN2 as 0..6; unary NEG..TAN,
//             ABS..CBRT as 0..13
//   bit 6     the terminal is a constant (value in y) rather than a feature
//   bit 7     "active": the subtree this instruction completes holds a
//             constant (only such instructions carry derivatives back)
//   bits 8-31 feature index, or the constant's slot
//   y         a constant's float bits; for an inactive instruction, the
//             index of the first instruction of the subtree it completes
//   z         up to 8 unary functions applied, in order, to the result of
//             the instruction (4 bits each from the lowest: unary function
//             index + 1; 0 ends the chain), so that a unary function costs no
//             dispatch of its own
//   w         (active instructions, in the adjoint's compile only) bits
//             0..25: index + 1 of the next active instruction its reverse
//             walk visits (0: none); bits 26..31: the subtrees without a
//             constant it skips before that one
// ---------------------------------------------------------------------------
enum : uint32_t { kPush = 0, kFold = 1, kBin = 2, kUn = 3 };
constexpr uint32_t kConstBit = 64u;
constexpr uint32_t kActive = 128u;
constexpr uint32_t kNextBits = 26u;
constexpr uint32_t kNextMask = (1u << kNextBits) - 1u;
constexpr int64_t kMaxAdjointLen = int64_t{1} << 25;   // program length the reverse links can address

GP_HD uint32_t enc(uint32_t cls, uint32_t fn, uint32_t is_const, uint32_t arg) {
    return cls | (fn << 2) | (is_const << 6) | (arg << 8);
}

// ---------------------------------------------------------------------------
// Register-resident arrays.  The compiler keeps a small local array in
// VGPRs, indexed by a wave-uniform value through M0-relative addressing,
// only when each array is a separate plain local; the R per-row copies are
// therefore spelled out one by one.
// ---------------------------------------------------------------------------
#define GP_ARRAYS(name, n) float name##0[n], name##1[n], name##2[n], name##3[n]
#define GP_PUT(name, idx, v)                         \
    do {                                             \
        name##0[idx] = v[0];                         \
        if constexpr (R > 1) name##1[idx] = v[1];    \
        if constexpr (R > 2) name##2[idx] = v[2];    \
        if constexpr (R > 3) name##3[idx] = v[3];    \
    } while (0)
#define GP_GET(name, idx, v)                         \
    do {                                             \
        v[0] = name##0[idx];                         \
        if constexpr (R > 1) v[1] = name##1[idx];    \
        if constexpr (R > 2) v[2] = name##2[idx];    \
        if constexpr (R > 3) v[3] = name##3[idx];    \
    } while (0)

// Uniform loads of read-only data through the scalar data cache: the pointer
// is cast to the constant address space so the compiler issues s_load.
template <typename T>
__device__ __forceinline__ T ldu(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

// Stack slots: slots below kStackRegs live in VGPRs, slots from kStackRegs
// on in a per-wavefront LDS area; register slot kStackRegs is a sink for the
// speculative writes of those deeper slots (see k_eval).  Slot 0 is never
// read, so a full stack of GP_MAX_STACK values uses slots 1 .. GP_MAX_STACK-1.
constexpr int kStackRegs = 15;
constexpr int kStackLds = GP_MAX_STACK - kStackRegs;

// Tables of the correctly rounded sin, cos and log (gp_crmath.h): staged in
// LDS by the evaluation and adjoint kernels, read from global memory
// elsewhere.
struct MathTabs {
    const crm::SinCosEntry* sc;
    const crm::LogEntry* lg;
};
__device__ __forceinline__ MathTabs global_tabs() { return MathTabs{crm::kSinCosTab, crm::kLogTab}; }

// The kernel-resident copies (one per block, filled before its first use).
struct MathTabsLds {
    crm::LogEntry lg[128];       // (at offset 0: its entries' address is the index alone)
    crm::SinCosEntry sc[128];    // (at 2 KB: the offset merges into the index's mask)
};
__device__ __forceinline__ MathTabs stage_tabs(MathTabsLds& lds) {
    for (int i = threadIdx.x; i < 128; i += blockDim.x) lds.sc[i] = crm::kSinCosTab[i];
    for (int i = threadIdx.x; i < 128; i += blockDim.x) lds.lg[i] = crm::kLogTab[i];
    __syncthreads();
    return MathTabs{lds.sc, lds.lg};
}

// Protected operators (reading of Sec. III-C3's function set: the gplearn
// convention).  Comparisons are written so that NaN takes the protected arm.
__device__ __forceinline__ float op_div(float a, float b) {
    return fabsf(b) > GP_PROTECT_EPS ? a / b : 1.0f;
}
__device__ __forceinline__ float op_log(float a, const MathTabs& mt, const crm::LogK& K) {
    // (evaluated on every lane, the protected ones included, so that the
    // protection is a select rather than a branch)
    const float l = crm::log_cr(fabsf(a), mt.lg, K);
    return fabsf(a) > GP_PROTECT_EPS ? l : 0.0f;
}

// The same on the R rows of a lane, with one branch, rarely taken, for the
// exception-table lookups of all the rows instead of one per row: fewer
// scalar instructions, but the rows' results and inputs are held together.
// The evaluation kernel goes row by row (the extra registers cost it an
// occupancy step); the adjoint kernel, with registers to spare at its
// occupancy, takes this form.
template <int R>
__device__ __forceinline__ void log_rows(float (&t)[R], const MathTabs& mt) {
    const crm::LogK K = crm::log_k();   // (once for the R rows)
    float f[R];
    bool near[R];
    bool any = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const double y = crm::log_double(fabsf(t[j]), mt.lg, K);   // (finite for inf and NaN)
        f[j] = static_cast<float>(y);
        near[j] = crm::near_boundary(y);
        any |= near[j];
    }
    if (any) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (near[j]) f[j] = crm::exception(crm::kLogExc, crm::kLogExcN, crm::fbits(fabsf(t[j])), f[j]);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const float a = fabsf(t[j]);
        const float l = a <= 0x1.fffffep+127f ? f[j] : a;   // +inf (and NaN) unchanged
        t[j] = a > GP_PROTECT_EPS ? l : 0.0f;
    }
}

// sqrt|a|, correctly rounded: in double from the hardware reciprocal square
// root y (relative error e below 2^-22) by two Newton steps on s = d y with
// h = y / 2 held fixed (the error goes e -> 1.5 e^2 -> about 1.5 e^3), then
// rounded to float.  A float's square root lies at least 2^-51 (relative)
// from every float rounding boundary (a - m^2 is a nonzero multiple of the
// least bit of m^2 for a midpoint m), so the double result, within 2^-53,
// rounds as the exact one does.  Zeros and infinity are passed through (the
// steps would give NaN there); NaN stays NaN.
__device__ __forceinline__ float op_sqrt(float a) {
    const double d = static_cast<double>(fabsf(a));
    const double y = __builtin_amdgcn_rsq(d);
    const double h = 0.5 * y;
    double s = d * y;
    s = fma(fma(-s, s, d), h, s);
    s = fma(fma(-s, s, d), h, s);
    // class mask: +0 (bit 6) or +inf (bit 9)
    return __builtin_amdgcn_class(d, 0x240) ? fabsf(a) : static_cast<float>(s);
}
__device__ __forceinline__ float op_inv(float a) {
    return fabsf(a) > GP_PROTECT_EPS ? 1.0f / a : 0.0f;
}

// t = sin t (is_cos false) or cos t on the R rows of a lane: the common
// path on every row, then one branch, rarely taken, for the rows with
// |t| >= 2^20, inf or NaN
template <int R>
__device__ __forceinline__ void sincos_rows(bool is_cos, float (&t)[R], const MathTabs& mt) {
    const crm::SinCosK K = crm::sincos_k(is_cos);   // (once for the R rows)
    float f[R];
    bool rare = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        f[j] = crm::sincos_common(t[j], is_cos, mt.sc, K);
        rare |= crm::sincos_rare_input(t[j]);
    }
    if (rare) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (crm::sincos_rare_input(t[j])) f[j] = crm::sincos_rare(t[j], is_cos, mt.sc, K);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) t[j] = f[j];
}

// a = a (op) b for the wider binary functions (MAX, MIN, ATAN2 as 4..6)
template <int R>
__device__ __forceinline__ void apply_binary_wide(uint32_t fn, float (&a)[R], const float (&b)[R]) {
    // max / min ignore a NaN operand; on equal operands the sign bits are
    // combined so that -0 orders below +0 whatever order fmaxf takes them in
    if (fn == 4) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float m = fmaxf(a[j], b[j]);
            a[j] = a[j] == b[j] ? __int_as_float(__float_as_int(a[j]) & __float_as_int(b[j])) : m;
        }
    } else if (fn == 5) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float m = fminf(a[j], b[j]);
            a[j] = a[j] == b[j] ? __int_as_float(__float_as_int(a[j]) | __float_as_int(b[j])) : m;
        }
    } else {
#pragma unroll
        for (int j = 0; j < R; ++j) a[j] = atan2f(a[j], b[j]);
    }
}

// t = f(t) for the wider unary functions (ABS..CBRT as 6..13)
template <int R>
__device__ __forceinline__ void apply_unary_wide(uint32_t fn, float (&t)[R]) {
    switch (fn) {
    case 6:
#pragma unroll
        for (int j = 0; j < R; ++j) t[j] = fabsf(t[j]);
        break;
    case 7:
#pragma unroll
        for (int j = 0; j < R; ++j) t[j] = expf(t[j]);
        break;
    case 8:
#pragma unroll
        for (int j = 0; j < R; ++j) t[j] = op_inv(t[j]);
        break;
    case 9:
#pragma unroll
        for (int j = 0; j < R; ++j) t[j] = t[j] * t[j];
        break;
    case 10:
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float q = t[j] * t[j];
            t[j] = q * t[j];
        }
        break;
    case 11:
#pragma unroll
        for (int j = 0; j < R; ++j) t[j] = tanhf(t[j]);
        break;
    case 12:
#pragma unroll
        for (int j = 0; j < R; ++j) t[j] = atanf(t[j]);
        break;
    default:
#pragma unroll
        for (int j = 0; j < R; ++j) t[j] = cbrtf(t[j]);
        break;
    }
}

// a = a (op) b for the binary function index fn (ADD, SUB, MUL, DIV first,
// then the wider set)
template <int R>
__device__ __forceinline__ void apply_binary(uint32_t fn, float (&a)[R], const float (&b)[R]) {
    if (fn >= 4) {
        apply_binary_wide<R>(fn, a, b);
    } else if (fn < 2) {
        if (fn == 0) {
#pragma unroll
            for (int j = 0; j < R; ++j) a[j] = a[j] + b[j];
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) a[j] = a[j] - b[j];
        }
    } else {
        if (fn == 2) {
#pragma unroll
            for (int j = 0; j < R; ++j) a[j] = a[j] * b[j];
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) a[j] = op_div(a[j], b[j]);
        }
    }
}

// t = f(t) for the unary function index fn (NEG, LOG, SQRT, SIN, COS, TAN
// first, then the wider set)
// (LOG_ROWS: the protected log by log_rows rather than row by row)
template <int R, bool LOG_ROWS = false>
__device__ __forceinline__ void apply_unary(uint32_t fn, float (&t)[R], const MathTabs& mt) {
    if (fn >= 6) {
        apply_unary_wide<R>(fn, t);
    } else if (fn < 3) {
        if (fn == 0) {
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = -t[j];
        } else if (fn == 1) {
            if constexpr (LOG_ROWS) {
                log_rows<R>(t, mt);
            } else {
                const crm::LogK K = crm::log_k();   // (once for the R rows)
#pragma unroll
                for (int j = 0; j < R; ++j) t[j] = op_log(t[j], mt, K);
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = op_sqrt(t[j]);
        }
    } else {
        if (fn == 3) {
            sincos_rows<R>(false, t, mt);
        } else if (fn == 4) {
            sincos_rows<R>(true, t, mt);
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = tanf(t[j]);
        }
    }
}

// ---------------------------------------------------------------------------
// k_compile: one lane per program.  Scans the prefix list right to left (the
// evaluation order of Sec. III-A) and emits instructions in that order.  A
// terminal at position i is the first operand of the function at i-1 exactly
// when that function is binary (its first operand starts right after it), so
// such pairs become one kFold instruction; a unary function is chained onto
// the instruction before it.  A shadow stack (in LDS, one column per lane)
// tracks, for each value on the evaluation stack, the first instruction of
// the subtree that produced it, whether that subtree holds a constant, and
// whether it holds nothing but constants.  With `fold`, a subtree of
// constants only is evaluated here, once, by the same float32 functions the
// evaluation kernel applies per row (so every row would get these very
// bits), and its instructions are replaced by one push of the result.
// ---------------------------------------------------------------------------
constexpr uint32_t kShStartMask = 0x3fffffffu;   // shadow entry: start | const-only << 30 | active << 31

__global__ __launch_bounds__(kBlock) void k_compile(PopView pop, uint4* __restrict__ code,
                                                     int32_t* __restrict__ clen, int fold) {
    __shared__ uint32_t shadow[GP_MAX_STACK][kBlock];
    __shared__ float shadow_v[GP_MAX_STACK][kBlock];   // value of a const-only entry
    const int32_t p = static_cast<int32_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= pop.P) return;
    const int64_t off = pop.prog_off[p];
    const int32_t L = pop.len[p];
    const uint32_t* pn = pop.nodes + off;
    const float* pc = pop.consts + pop.const_off[p];
    uint4* out = code + off;
    uint32_t* sh = &shadow[0][threadIdx.x];   // entry h at sh[h * kBlock]
    float* shv = &shadow_v[0][threadIdx.x];
    int h = 0;                                // shadow stack height
    int32_t k = 0;                            // instructions emitted
    uint4 pend = make_uint4(0u, 0u, 0u, 0u);  // the last instruction, still open for a unary chain
    int chain = -1;                           // unary functions chained on it (-1: none pending)
    for (int32_t i = L - 1; i >= 0; --i) {
        const uint32_t w = pn[i];
        const uint32_t op = w & 0xffu;
        const uint32_t arg = w >> 8;
        const int top_i = min(max(h - 1, 0), GP_MAX_STACK - 1);
        const int ar = arity(op);
        if (ar == 1 && fold && h >= 1 && ((sh[top_i * kBlock] >> 30) & 1u)) {
            // unary of a constant: the pending instruction is that constant's push
            float t[1] = {shv[top_i * kBlock]};
            apply_unary<1>(unary_index(op), t, global_tabs());
            shv[top_i * kBlock] = t[0];
            pend.y = __float_as_uint(t[0]);
            continue;
        }
        if (ar == 1 && chain >= 0 && chain < 8) {
            // a unary function applied to the pending instruction's result:
            // same subtree start and activity as its operand
            pend.z |= (unary_index(op) + 1u) << (4 * chain);
            ++chain;
            continue;
        }
        uint32_t x, start, active, konst = 0u;
        float kval = 0.0f;
        uint2 xy;
        if (op <= GP_OP_CONST) {
            const uint32_t is_c = op == GP_OP_CONST ? 1u : 0u;
            const uint32_t farg = arg;   // feature index, or constant slot (used by the adjoint)
            const uint32_t prev = i >= 1 ? (pn[i - 1] & 0xffu) : 0u;
            if (i >= 1 && i != L - 1 && arity(prev) == 2) {
                const uint32_t top = sh[top_i * kBlock];    // the second operand
                start = top & kShStartMask;
                if (fold && is_c && ((top >> 30) & 1u)) {
                    // constant op constant: evaluated here
                    float a[1] = {pc[arg]};
                    const float b[1] = {shv[top_i * kBlock]};
                    apply_binary<1>(binary_index(prev), a, b);
                    x = enc(kPush, 0, 1u, 0u);
                    active = 1u;
                    konst = 1u;
                    kval = a[0];
                    k = static_cast<int32_t>(start);   // drop the operand's instructions
                    chain = -1;
                } else {
                    x = enc(kFold, binary_index(prev), is_c, farg);
                    active = is_c | (top >> 31);
                }
                --h;
                --i;
            } else {
                x = enc(kPush, 0, is_c, farg);
                start = static_cast<uint32_t>(k);
                active = is_c;
                konst = is_c;
                kval = is_c ? pc[arg] : 0.0f;
            }
            xy = (is_c || konst) ? make_uint2(x | kActive, __float_as_uint(konst ? kval : pc[arg]))
                                 : make_uint2(x | (active ? kActive : 0u), start);
        } else if (ar == 2) {
            const int i1 = min(max(h - 1, 0), GP_MAX_STACK - 1), i2 = min(max(h - 2, 0), GP_MAX_STACK - 1);
            const uint32_t first = sh[i1 * kBlock];      // top: the first operand
            const uint32_t second = sh[i2 * kBlock];     // evaluated before it
            start = second & kShStartMask;
            h -= 2;
            if (fold && ((first >> 30) & 1u) && ((second >> 30) & 1u)) {
                float a[1] = {shv[i1 * kBlock]};
                const float b[1] = {shv[i2 * kBlock]};
                apply_binary<1>(binary_index(op), a, b);
                x = enc(kPush, 0, 1u, 0u);
                active = 1u;
                konst = 1u;
                kval = a[0];
                k = static_cast<int32_t>(start);
                chain = -1;
                xy = make_uint2(x | kActive, __float_as_uint(kval));
            } else {
                x = enc(kBin, binary_index(op), 0, 0);
                active = (first >> 31) | (second >> 31);
                xy = make_uint2(x | (active ? kActive : 0u), start);
            }
        } else {
            // a unary function with a full chain before it: its own instruction
            const uint32_t top = sh[top_i * kBlock];
            x = enc(kUn, unary_index(op), 0, 0);
            start = top & kShStartMask;
            active = top >> 31;
            --h;
            xy = make_uint2(x | (active ? kActive : 0u), start);
        }
        if (chain >= 0) out[k - 1] = pend;
        pend = make_uint4(xy.x, xy.y, 0u, 0u);
        chain = 0;
        // (valid programs keep 1 <= h <= GP_MAX_STACK; the clamps only keep an
        // invalid one inside this array)
        h = max(h, 0);
        const int hi = min(h, GP_MAX_STACK - 1);
        sh[hi * kBlock] = start | (konst << 30) | (active << 31);
        shv[hi * kBlock] = kval;
        ++h;
        ++k;
    }
    if (chain >= 0) out[k - 1] = pend;
    clen[p] = k;
    // the adjoint's reverse walk (its compile is the one without folding),
    // from the last instruction down: an inactive instruction stands for its
    // whole subtree (skipped, one stack entry); each active one is linked to
    // the next active one and counts the skips between them.  (Indices stay
    // below 2^26 for programs the adjoint accepts; skips never exceed the
    // stack depth, below 2^6.)
    if (fold) return;
    int32_t last = -1;
    uint32_t skips = 0u;
    for (int32_t q = k - 1; q >= 0;) {
        const uint4 ins = out[q];
        if (!(ins.x & kActive)) {
            ++skips;
            q = min(static_cast<int32_t>(ins.y), q) - 1;   // (the clamp only guards a malformed program)
            continue;
        }
        if (last >= 0) out[last].w = (static_cast<uint32_t>(q + 1) & kNextMask) | (min(skips, 63u) << kNextBits);
        last = q;
        skips = 0u;
        --q;
    }
    if (last >= 0) out[last].w = 0u;
}

// ---------------------------------------------------------------------------
// The evaluation kernel's instruction stream (k_compile_eval): one uint4 per
// instruction, in execution order, each instruction's stack slots fixed by
// the pre-pass, so the kernel keeps no stack pointer.
//   x bits 0-7    opcode (below)
//   x bits 8-15   slot the kernel stores the current top into before the
//                 instruction: for a push, the slot of the entry it covers;
//                 for every other instruction the sink slot kEvalRegs, which
//                 is never read (one store per instruction keeps the
//                 register array in place)
//   x bits 16-23  slot of a binary function's second operand (kIBin); the
//                 LDS slot a deep push covers (kIDeep)
//   y             a constant's float bits (kIPushC, kIFoldC), a feature
//                 index (kIPushX, kIFoldX) or the slot a copy reads (kIPushS)
//   z             up to 8 unary functions applied, in order, to the
//                 instruction's result (4 bits each from the lowest: unary
//                 index + 1; 0 ends the chain), so that a unary function
//                 costs no dispatch of its own
// Stack entries are numbered from the bottom; the top entry lives in
// registers and entry e below it in slot e.  Slots from kEvalRegs on live in
// LDS; the instructions that reach them carry kIDeep.
//
// A user function (Sec. V: custom function sets) is expanded in place: its
// arguments are evaluated as usual, its definition's argument references
// become kIPushS copies of the argument entries, and once the definition has
// left its value on top, the arguments below it are simply forgotten (the
// next push overwrites their slots).  A user loss (GP_METRIC_USER_i) is the
// same expansion around the whole program: kIPushY pushes the row's target
// first, and the loss function's definition runs on (output, target) last.
// These stacks reach past the program's own GP_MAX_STACK, into LDS slots
// kEvalLds .. kEvalLdsUser-1, which launches that may meet them provide.
// ---------------------------------------------------------------------------
enum : uint32_t {
    kIPushX = 0,    // push feature
    kIPushC = 1,    // push constant
    kIBin = 2,      // + binary index: top = top (op) slot
    kIFoldX = 9,    // + binary index: top = feature (op) top
    kIFoldC = 16,   // + binary index: top = constant (op) top
    kIUn = 23,      // + unary index: top = f(top)
    kIPushS = 40,   // push a copy of the entry in slot y (register or LDS)
    kIPushY = 41,   // push the row's target
    kIDeep = 64     // with kIPushX, kIPushC, kIPushS, kIBin: the slot x
                    // bits 16-23 names lives in LDS
};
constexpr int kEvalSlots = GP_MAX_STACK - 1;   // entries below the top
constexpr int kEvalRegs = 15;                  // slots held in VGPRs (plus the sink)
constexpr int kEvalLds = kEvalSlots - kEvalRegs;
// with user functions or a user loss: the target below the program, and a
// definition's own GP_USER_MAX_STACK values above its arguments
constexpr int kEvalSlotsUser = GP_MAX_STACK + GP_USER_MAX_STACK;
constexpr int kEvalLdsUser = kEvalSlotsUser - kEvalRegs;
constexpr int kCompileDepth = kEvalSlotsUser + 1;   // entries the compiler tracks

__device__ __forceinline__ uint32_t ins_x(uint32_t op, uint32_t wslot, uint32_t rslot) {
    return op | (wslot << 8) | (rslot << 16);
}

// k_compile_eval: one lane per program; the same right-to-left scan as
// k_compile, emitting the stream above.  A terminal that is a binary
// function's first operand is fused with it; a unary function is chained
// onto the instruction before it; a subtree of constants only is evaluated
// here, once, by the same float32 functions the kernel applies per row, and
// replaced by one push of its value.  User functions are expanded from
// `ud`; loss_fn >= 0 wraps the program in the user loss (GP_OP_USER2 +
// loss_fn) of (output, target).
__global__ __launch_bounds__(kBlock) void k_compile_eval(PopView pop, uint4* __restrict__ code,
                                                          int32_t* __restrict__ clen, UserDefs ud,
                                                          int32_t loss_fn, int32_t ex_mul, int32_t ex_add) {
    __shared__ uint32_t shadow[kCompileDepth][kBlock];   // start | const-only << 31
    __shared__ float shadow_v[kCompileDepth][kBlock];    // value of a const-only entry
    const int32_t p = static_cast<int32_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= pop.P) return;
    const int64_t off = pop.prog_off[p];
    const int32_t L = pop.len[p];
    const uint32_t* pn = pop.nodes + off;
    const float* pc = pop.consts + pop.const_off[p];
    uint4* out = code + off * ex_mul + static_cast<int64_t>(p) * ex_add;
    uint32_t* sh = &shadow[0][threadIdx.x];   // entry h at sh[h * kBlock]
    float* shv = &shadow_v[0][threadIdx.x];
    int h = 0;                                // entries on the stack
    int32_t k = 0;                            // instructions emitted
    int chain = 0;                            // unary functions chained on out[k-1]
    const uint32_t sink = static_cast<uint32_t>(kEvalRegs);
    auto clampe = [](int e) { return min(max(e, 0), kCompileDepth - 1); };
    // a push of constant v as entry e
    auto push_c = [&](int e, float v) {
        const uint32_t slot = static_cast<uint32_t>(max(e - 1, 0));
        return slot >= sink ? make_uint4(ins_x(kIPushC | kIDeep, sink, slot), __float_as_uint(v), 0u, 0u)
                            : make_uint4(ins_x(kIPushC, slot, 0u), __float_as_uint(v), 0u, 0u);
    };
    // a push of the value of entry src as entry e
    auto push_s = [&](int e, int src) {
        const uint32_t slot = static_cast<uint32_t>(max(e - 1, 0));
        const uint32_t rs = static_cast<uint32_t>(clampe(src));
        return slot >= sink ? make_uint4(ins_x(kIPushS | kIDeep, sink, slot), rs, 0u, 0u)
                            : make_uint4(ins_x(kIPushS, slot, 0u), rs, 0u, 0u);
    };
    auto emit = [&](uint4 ins) {
        out[k++] = ins;
        chain = 0;
    };
    // The item source: the program right to left; while a user function is
    // expanded, its definition right to left.  (i: next program position;
    // uf: the function being expanded or -1, di its next position, call_h
    // the stack height when it began, call_ar its arity.)
    int32_t i = L - 1;
    int uf = -1, di = 0, call_h = 0, call_ar = 0;
    bool loss_pending = loss_fn >= 0;
    if (loss_pending) {
        // entry 0: the target, under the program's value
        emit(make_uint4(ins_x(kIPushY, 0u, 0u), 0u, 0u, 0u));
        sh[0] = 0u;
        h = 1;
    }
    for (;;) {
        uint32_t w;
        bool in_def;
        if (uf >= 0) {
            if (di < 0) {
                // end of the expansion: the value replaces the arguments
                const int base = max(call_h - call_ar, 0);
                sh[clampe(base) * kBlock] = sh[clampe(base) * kBlock] & 0x7fffffffu;   // the deepest argument's start
                h = base + 1;
                uf = -1;
                continue;
            }
            w = ud.nodes[uf][di];
            in_def = true;
        } else {
            if (i < 0) {
                if (!loss_pending) break;
                loss_pending = false;
                uf = kUserFns / 2 + loss_fn;   // the two-argument user functions follow the one-argument ones
                di = ud.len[uf] - 1;
                call_h = h;
                call_ar = 2;
                continue;
            }
            w = pn[i];
            in_def = false;
        }
        const uint32_t op = w & 0xffu;
        const uint32_t arg = w >> 8;
        if (!in_def && is_user_op(op)) {
            uf = static_cast<int>(op - GP_OP_USER1);
            di = ud.len[uf] - 1;
            call_h = h;
            call_ar = arity(op);
            --i;
            continue;
        }
        if (in_def && op == GP_OP_VAR) {
            // argument `arg` of the function: entry call_h - 1 - arg
            const int e = clampe(h);
            emit(push_s(e, call_h - 1 - static_cast<int>(arg)));
            sh[e * kBlock] = static_cast<uint32_t>(k - 1);
            ++h;
            --di;
            continue;
        }
        // position and the item before it in the same source (a terminal
        // fuses only with a built-in binary function of its own source)
        const int32_t pos = in_def ? di : i;
        const int32_t last = in_def ? ud.len[uf] - 1 : L - 1;
        const uint32_t prev = pos >= 1 ? ((in_def ? ud.nodes[uf][pos - 1] : pn[pos - 1]) & 0xffu) : 0u;
        const float cval = op == GP_OP_CONST ? (in_def ? ud.consts[uf][arg & (GP_USER_MAX_CONSTS - 1)] : pc[arg])
                                             : 0.0f;
        auto advance = [&](int n) {
            if (in_def) di -= n;
            else i -= n;
        };
        const int ar = arity(op);
        const int top = clampe(h - 1);
        if (ar == 1) {
            if (h >= 1 && (sh[top * kBlock] >> 31)) {
                // a unary function of a constant: its push (the last
                // instruction) takes the value
                float t[1] = {shv[top * kBlock]};
                apply_unary<1>(unary_index(op), t, global_tabs());
                shv[top * kBlock] = t[0];
                if (k >= 1) out[k - 1].y = __float_as_uint(t[0]);
            } else if (k >= 1 && chain < 8) {
                out[k - 1].z |= (unary_index(op) + 1u) << (4 * chain);
                ++chain;
            } else {
                emit(make_uint4(ins_x(kIUn + unary_index(op), sink, 0u), 0u, 0u, 0u));
            }
            advance(1);
            continue;
        }
        if (ar == 0) {
            const uint32_t is_c = op == GP_OP_CONST ? 1u : 0u;
            if (pos >= 1 && pos != last && is_builtin_binary(prev) && h >= 1) {
                // first operand of the binary function before it; the top is the second
                const uint32_t fn = binary_index(prev);
                const uint32_t e2 = sh[top * kBlock];
                if (is_c && (e2 >> 31)) {
                    float a[1] = {cval};
                    const float b[1] = {shv[top * kBlock]};
                    apply_binary<1>(fn, a, b);
                    k = static_cast<int32_t>(e2 & 0x7fffffffu);   // drop the operand's instructions
                    emit(push_c(top, a[0]));
                    sh[top * kBlock] = static_cast<uint32_t>(k - 1) | (1u << 31);
                    shv[top * kBlock] = a[0];
                } else {
                    emit(is_c ? make_uint4(ins_x(kIFoldC + fn, sink, 0u), __float_as_uint(cval), 0u, 0u)
                              : make_uint4(ins_x(kIFoldX + fn, sink, 0u), arg, 0u, 0u));
                    sh[top * kBlock] = e2 & 0x7fffffffu;
                }
                advance(2);
                continue;
            }
            const int e = clampe(h);
            if (is_c) {
                emit(push_c(e, cval));
                sh[e * kBlock] = static_cast<uint32_t>(k - 1) | (1u << 31);
                shv[e * kBlock] = cval;
            } else {
                const uint32_t slot = static_cast<uint32_t>(max(e - 1, 0));
                emit(slot >= sink ? make_uint4(ins_x(kIPushX | kIDeep, sink, slot), arg, 0u, 0u)
                                  : make_uint4(ins_x(kIPushX, slot, 0u), arg, 0u, 0u));
                sh[e * kBlock] = static_cast<uint32_t>(k - 1);
            }
            ++h;
            advance(1);
            continue;
        }
        // binary, operands not fused: the first is the top (entry h-1), the
        // second the entry below it (slot h-2)
        const int e1 = clampe(h - 1), e2 = clampe(h - 2);
        const uint32_t first = sh[e1 * kBlock], second = sh[e2 * kBlock];
        const uint32_t fn = binary_index(op);
        if ((first >> 31) && (second >> 31)) {
            float a[1] = {shv[e1 * kBlock]};
            const float b[1] = {shv[e2 * kBlock]};
            apply_binary<1>(fn, a, b);
            k = static_cast<int32_t>(second & 0x7fffffffu);
            emit(push_c(e2, a[0]));
            sh[e2 * kBlock] = static_cast<uint32_t>(k - 1) | (1u << 31);
            shv[e2 * kBlock] = a[0];
        } else {
            const uint32_t slot = static_cast<uint32_t>(e2);
            emit(make_uint4(ins_x(kIBin + fn | (slot >= sink ? kIDeep : 0u), sink, slot), 0u, 0u, 0u));
            sh[e2 * kBlock] = second & 0x7fffffffu;
        }
        h = max(h - 1, 0);
        advance(1);
    }
    clen[p] = k;
}

// ---------------------------------------------------------------------------
// k_find_user: raises flag[0] (which the caller zeroes, k_zero_u32) if any
// of the n nodes is a user function.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_find_user(const uint32_t* __restrict__ nodes, int64_t n,
                                                       uint32_t* __restrict__ flag) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        if (is_user_op(nodes[i] & 0xffu)) flag[0] = 1u;
}

__global__ void k_zero_u32(uint32_t* __restrict__ p) { p[0] = 0u; }

// ---------------------------------------------------------------------------
// k_prepare: order programs by length (longest first) and reset the work
// counter.  One block; counting sort over min(len, kBins-1).
// ---------------------------------------------------------------------------
constexpr int kBins = 1024;

__global__ __launch_bounds__(1024) void k_prepare(const int32_t* __restrict__ len, int32_t P,
                                                   int32_t* __restrict__ order,
                                                   uint32_t* __restrict__ counter) {
    __shared__ int32_t start[kBins];
    const int tid = threadIdx.x;
    for (int b = tid; b < kBins; b += blockDim.x) start[b] = 0;
    __syncthreads();
    // key: kBins-1 - min(len, kBins-1), so longer programs come first
    for (int p = tid; p < P; p += blockDim.x) {
        const int key = kBins - 1 - min(max(len[p], 0), kBins - 1);
        atomicAdd(&start[key], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int b = 0; b < kBins; ++b) {
            const int32_t c = start[b];
            start[b] = run;
            run += c;
        }
        for (int q = 0; q < kQueues; ++q) counter[q * kQueueStride] = 0u;
    }
    __syncthreads();
    for (int p = tid; p < P; p += blockDim.x) {
        const int key = kBins - 1 - min(max(len[p], 0), kBins - 1);
        order[atomicAdd(&start[key], 1)] = p;
    }
}

// ---------------------------------------------------------------------------
// k_ystats: per chunk, float64 sums of the weights and of the shifted target
// (shift = y at the chunk's first row): S0 = sum w, S1 = sum w (y-K),
// S2 = sum w (y-K)^2, K.  One wavefront per chunk.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__global__ __launch_bounds__(kBlock) void k_ystats(DataView d, int64_t chunk, int32_t n_chunks,
                                                    double* __restrict__ ystat) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t c = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + (threadIdx.x >> 6);
    if (c >= n_chunks) return;
    const int64_t r0 = c * chunk;
    const int64_t r1 = min(r0 + chunk, d.N);
    const double K = static_cast<double>(d.y[r0]);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t r = r0 + lane; r < r1; r += kWave) {
        const double w = d.w ? static_cast<double>(d.w[r]) : 1.0;
        const double b = static_cast<double>(d.y[r]) - K;
        s0 += w;
        s1 += w * b;
        s2 += w * b * b;
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
        ystat[c * 4 + 0] = s0;
        ystat[c * 4 + 1] = s1;
        ystat[c * 4 + 2] = s2;
        ystat[c * 4 + 3] = K;
    }
}

// ---------------------------------------------------------------------------
// The evaluation kernel.
//   MODE 0: write every program output out[p * N + r]   (gp_evaluate)
//   MODE 1: accumulate the metric's float64 row sums per (program, chunk)
//           into part[(p * n_chunks + c) * KK + k]     (gp_fitness)
// R rows per lane; FREG > 0 keeps the tile's F <= FREG feature values in
// registers, FREG == 0 reads a feature from memory at each terminal.
// ---------------------------------------------------------------------------
template <int METRIC>
struct MetricTraits {
    static constexpr int K = (METRIC == GP_METRIC_PEARSON) ? 3 : 1;   // moments per row
    static constexpr int KK = (METRIC == GP_METRIC_PEARSON) ? 4 : 1;  // doubles per partial
};

// Row-slot helpers of the evaluation kernel: the R per-row copies of a
// register array are separate plain locals (GP_ARRAYS), indexed by a
// wave-uniform slot.
#define GP_ROWS(stmt)                  \
    _Pragma("unroll") for (int j = 0; j < R; ++j) { stmt; }

template <int R, int FREG, int MODE, int METRIC>
__global__ __launch_bounds__(kBlock) void k_eval(PopView pop, CodeView cv, DataView d, Sched s,
                                                  float* __restrict__ out,
                                                  double* __restrict__ part) {
    constexpr int K = MetricTraits<METRIC>::K;
    constexpr int KK = MetricTraits<METRIC>::KK;
    constexpr int FA = FREG > 0 ? FREG : 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t N = d.N;
    const int64_t ld = d.ld;
    const float* __restrict__ X = d.X;
    // stack slots beyond the registers: s.lds_slots * R * 64 floats per
    // wavefront of the block (dynamic LDS, sized at launch: kEvalLds, or
    // kEvalLdsUser when user functions may be expanded)
    extern __shared__ float ovf_all[];
    float* ovf = ovf_all + (threadIdx.x >> 6) * (s.lds_slots * R * kWave) + lane;
    __shared__ MathTabsLds tabs_lds;
    const MathTabs mt = stage_tabs(tabs_lds);

    // Work items: one queue per XCD.  Queue x holds the chunks c with
    // c % kQueues == x, chunk-major, each chunk's programs in LPT order
    // (longest first), so that a chunk's rows are read into one L2 while
    // every program walks them.  Blocks are dealt to the XCDs in turn, so
    // a block starts on queue blockIdx.x % kQueues; a wavefront whose queue
    // has run dry takes items from the next ones, and leaves once all are
    // dry.  A claim takes s.batch consecutive items.
    const int q0 = static_cast<int>(blockIdx.x % kQueues);
    for (int qi = 0; qi < kQueues;) {
        const int qx = (q0 + qi) % kQueues;
        const int64_t q_items = (static_cast<int64_t>(s.n_chunks) - qx + kQueues - 1) / kQueues * pop.P;
        uint32_t it32 = 0;
        if (lane == 0) it32 = atomicAdd(s.counter + qx * kQueueStride, static_cast<uint32_t>(s.batch));
        const int64_t it0 = static_cast<int64_t>(
            static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(it32))));
        if (it0 >= q_items) {   // this queue is dry: the next one
            ++qi;
            continue;
        }
        const int64_t it1 = min(it0 + static_cast<int64_t>(s.batch), q_items);
        for (int64_t it = it0; it < it1; ++it) {
        const int32_t cq = static_cast<int32_t>(it / pop.P);
        const int32_t k = static_cast<int32_t>(it - static_cast<int64_t>(cq) * pop.P);
        const int32_t c = cq * kQueues + qx;
        const int32_t p = ldu(s.order + k);
        const int64_t off = ldu(pop.prog_off + p);
        const int32_t CL = ldu(cv.eclen + p);
        const uint4* __restrict__ pcode = cv.ecode + off * cv.ex_mul + static_cast<int64_t>(p) * cv.ex_add;
        const int64_t r0 = static_cast<int64_t>(c) * s.chunk;
        const int64_t r1 = min(r0 + s.chunk, N);

        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
        double shift = 0.0, yshift = 0.0;
        if constexpr (METRIC == GP_METRIC_PEARSON) yshift = static_cast<double>(d.y[r0]);
        bool first_tile = true;

        for (int64_t base = r0; base < r1; base += kWave * R) {
            int64_t row[R];
            bool valid[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int64_t r = base + j * kWave + lane;
                valid[j] = r < r1;
                row[j] = valid[j] ? r : r1 - 1;
            }
            // feature tile in registers (one array per row slot)
            GP_ARRAYS(xa, FA);
            if constexpr (FREG > 0) {
#pragma unroll
                for (int f = 0; f < FREG; ++f) {
                    if (f < d.F) {
                        xa0[f] = X[f * ld + row[0]];
                        if constexpr (R > 1) xa1[f] = X[f * ld + row[1]];
                        if constexpr (R > 2) xa2[f] = X[f * ld + row[2]];
                        if constexpr (R > 3) xa3[f] = X[f * ld + row[3]];
                    }
                }
            }

            // ---- the stack machine (Sec. III-A order, compiled by k_compile_eval) ----
            // t[] is the top entry; entry e below it is slot e (VGPRs below
            // kEvalRegs, LDS from there on).  Each instruction first stores the
            // top into its store slot (the sink unless it pushes), so the
            // register array has one indexed write per instruction and is
            // never copied; every case then updates t[] in place.  The next
            // instruction is fetched one ahead by a vector load (in order
            // with the others, so its wait covers only the older loads; a
            // scalar load is waited for with every other one) and made
            // scalar where it is used.
            float t[R];
            GP_ROWS(t[j] = 0.0f);
            GP_ARRAYS(st, kEvalRegs + 1);
            uint4 nxt = pcode[0];
            for (int q = 0; q < CL; ++q) {
                const uint4 cur = nxt;
                nxt = pcode[q + 1];
                const uint32_t cx = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.x)));
                const uint32_t cy = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.y)));
                const uint32_t cz = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.z)));
                const uint32_t op = cx & 0xffu;
                const uint32_t wslot = (cx >> 8) & 0xffu;
                const uint32_t rslot = cx >> 16;
                GP_PUT(st, wslot, t);
                float v[R];   // a terminal's value
                // the feature cy (for kIPushX / kIFoldX)
#define GP_FEATURE()                                                          \
    do {                                                                      \
        if constexpr (FREG > 0) {                                             \
            v[0] = xa0[cy];                                                   \
            if constexpr (R > 1) v[1] = xa1[cy];                              \
            if constexpr (R > 2) v[2] = xa2[cy];                              \
            if constexpr (R > 3) v[3] = xa3[cy];                              \
        } else {                                                              \
            const float* __restrict__ col = X + static_cast<int64_t>(cy) * ld; \
            GP_ROWS(v[j] = col[row[j]]);                                      \
        }                                                                     \
    } while (0)
#define GP_BIN_CASES(BASE, LOAD)                                                        \
    case (BASE) + 0: { LOAD; GP_ROWS(t[j] = A0 + B0); } break;                          \
    case (BASE) + 1: { LOAD; GP_ROWS(t[j] = A0 - B0); } break;                          \
    case (BASE) + 2: { LOAD; GP_ROWS(t[j] = A0 * B0); } break;                          \
    case (BASE) + 3: { LOAD; GP_ROWS(t[j] = op_div(A0, B0)); } break;                   \
    case (BASE) + 4: case (BASE) + 5: case (BASE) + 6: {                                    \
        LOAD; float a_[R], b_[R]; GP_ROWS(a_[j] = A0; b_[j] = B0);                    \
        apply_binary_wide<R>(op - (BASE), a_, b_); GP_ROWS(t[j] = a_[j]);             \
    } break;
                switch (op) {
                case kIPushX: GP_FEATURE(); GP_ROWS(t[j] = v[j]); break;
                case kIPushC: {
                    const float cval = __uint_as_float(cy);
                    GP_ROWS(t[j] = cval);
                } break;
                case kIPushX | kIDeep: {
                    GP_FEATURE();
                    GP_ROWS(ovf[((rslot - kEvalRegs) * R + j) * kWave] = t[j]);
                    GP_ROWS(t[j] = v[j]);
                } break;
                case kIPushC | kIDeep: {
                    const float cval = __uint_as_float(cy);
                    GP_ROWS(ovf[((rslot - kEvalRegs) * R + j) * kWave] = t[j]);
                    GP_ROWS(t[j] = cval);
                } break;
                case kIPushS:
                case kIPushS | kIDeep: {
                    // (the covered entry is stored first: a copy of the
                    // entry just covered reads it back)
                    if (op & kIDeep) GP_ROWS(ovf[((rslot - kEvalRegs) * R + j) * kWave] = t[j]);
                    if (cy < static_cast<uint32_t>(kEvalRegs)) {
                        GP_GET(st, cy, v);
                    } else {
                        GP_ROWS(v[j] = ovf[((cy - kEvalRegs) * R + j) * kWave]);
                    }
                    GP_ROWS(t[j] = v[j]);
                } break;
                case kIPushY: GP_ROWS(t[j] = d.y[row[j]]); break;
#define A0 t[j]
#define B0 v[j]
                GP_BIN_CASES(kIBin, GP_GET(st, rslot, v))
                GP_BIN_CASES(kIBin | kIDeep, GP_ROWS(v[j] = ovf[((rslot - kEvalRegs) * R + j) * kWave]))
#undef A0
#undef B0
#define A0 v[j]
#define B0 t[j]
                GP_BIN_CASES(kIFoldX, GP_FEATURE())
                GP_BIN_CASES(kIFoldC, const float cval = __uint_as_float(cy); GP_ROWS(v[j] = cval))
#undef A0
#undef B0
                default: apply_unary<R>(op - kIUn, t, mt); break;
                }
                // the unary functions chained on this instruction
                for (uint32_t ch = cz; ch != 0u; ch >>= 4) apply_unary<R>((ch & 15u) - 1u, t, mt);
#undef GP_BIN_CASES
#undef GP_FEATURE
            }

            if constexpr (MODE == 0) {
                float* __restrict__ o = out + static_cast<int64_t>(p) * N;
#pragma unroll
                for (int j = 0; j < R; ++j)
                    if (valid[j]) o[row[j]] = t[j];
            } else {
                if constexpr (METRIC == GP_METRIC_PEARSON) {
                    if (first_tile) shift = static_cast<double>(__shfl(t[0], 0, kWave));
                }
                first_tile = false;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const float yv = d.y[row[j]];
                    const double wv = d.w ? static_cast<double>(d.w[row[j]]) : 1.0;
                    if constexpr (METRIC == GP_METRIC_MSE || METRIC == GP_METRIC_RMSE) {
                        const double e = static_cast<double>(t[j]) - static_cast<double>(yv);
                        const double l = e * e;
                        const double term = wv * l;
                        acc0 += valid[j] ? term : 0.0;
                    } else if constexpr (METRIC == GP_METRIC_MAE) {
                        const double e = static_cast<double>(t[j]) - static_cast<double>(yv);
                        const double term = wv * fabs(e);
                        acc0 += valid[j] ? term : 0.0;
                    } else if constexpr (METRIC == GP_METRIC_USER_0) {
                        // a user loss: the stream already ends in the row loss
                        (void)yv;
                        const double term = wv * static_cast<double>(t[j]);
                        acc0 += valid[j] ? term : 0.0;
                    } else if constexpr (METRIC == GP_METRIC_LOGLOSS) {
                        const float z = t[j];
                        const float t1 = fmaxf(z, 0.0f);
                        const float t2 = yv * z;
                        const float t3 = t1 - t2;
                        const float t5 = log1pf(expf(-fabsf(z)));
                        const double term = wv * static_cast<double>(t3 + t5);
                        acc0 += valid[j] ? term : 0.0;
                    } else {  // PEARSON: shifted first and second moments
                        const double a = static_cast<double>(t[j]) - shift;
                        const double bb = static_cast<double>(yv) - yshift;
                        const double wa = wv * a;
                        acc0 += valid[j] ? wa : 0.0;
                        acc1 += valid[j] ? wa * a : 0.0;
                        acc2 += valid[j] ? wa * bb : 0.0;
                    }
                }
            }
        }
        if constexpr (MODE == 1) {
            acc0 = wave_sum(acc0);
            if constexpr (K > 1) {
                acc1 = wave_sum(acc1);
                acc2 = wave_sum(acc2);
            }
            if (lane == 0) {
                double* dst = part + (static_cast<int64_t>(p) * s.n_chunks + c) * KK;
                dst[0] = acc0;
                if constexpr (K > 1) {
                    dst[1] = acc1;
                    dst[2] = acc2;
                    dst[3] = shift;
                }
            }
        }
        }
    }
}
#undef GP_ROWS

// ---------------------------------------------------------------------------
// k_finalize: merge each program's chunk partials in a fixed order (float64)
// and apply the metric.  One wavefront per program.
// ---------------------------------------------------------------------------
struct Moments {  // weighted count, means and centred second moments
    double W, ma, mb, Maa, Mbb, Mab;
};

__device__ __forceinline__ Moments merge(const Moments& x, const Moments& y) {
    // pairwise update (Chan, Golub, LeVeque) for weighted means and
    // co-moments
    if (!(x.W > 0.0)) return y;
    if (!(y.W > 0.0)) return x;
    Moments m;
    m.W = x.W + y.W;
    const double da = y.ma - x.ma, db = y.mb - x.mb;
    const double f = x.W * y.W / m.W;
    m.ma = x.ma + da * (y.W / m.W);
    m.mb = x.mb + db * (y.W / m.W);
    m.Maa = x.Maa + y.Maa + da * da * f;
    m.Mbb = x.Mbb + y.Mbb + db * db * f;
    m.Mab = x.Mab + y.Mab + da * db * f;
    return m;
}

__device__ __forceinline__ Moments shfl_moments(const Moments& m, int src) {
    Moments r;
    r.W = __shfl_xor(m.W, src, kWave);
    r.ma = __shfl_xor(m.ma, src, kWave);
    r.mb = __shfl_xor(m.mb, src, kWave);
    r.Maa = __shfl_xor(m.Maa, src, kWave);
    r.Mbb = __shfl_xor(m.Mbb, src, kWave);
    r.Mab = __shfl_xor(m.Mab, src, kWave);
    return r;
}

// stats (nullable) receives per program: [0] sum of weights W, [1] mean of
// yhat, [2] mean of y, [3] sum w (yhat - mean)^2, [4] sum w (y - mean)^2,
// [5] sum w (yhat - mean)(y - mean), [6] the metric in float64 (Pearson: the
// signed r), [7] unused.
constexpr int kStats = 8;

template <int METRIC>
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ part,
                                                      const double* __restrict__ ystat,
                                                      int32_t n_chunks, int32_t P, int64_t N,
                                                      int has_w, float* __restrict__ fitness,
                                                      double* __restrict__ stats) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t p = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + (threadIdx.x >> 6);
    if (p >= P) return;
    if constexpr (METRIC == GP_METRIC_PEARSON) {
        Moments m{0, 0, 0, 0, 0, 0};
        for (int c = lane; c < n_chunks; c += kWave) {
            const double* q = part + (p * n_chunks + c) * 4;
            const double* ys = ystat + static_cast<int64_t>(c) * 4;
            Moments x;
            x.W = ys[0];
            const double Sa = q[0], Saa = q[1], Sab = q[2], Ka = q[3];
            const double Sb = ys[1], Sbb = ys[2], Kb = ys[3];
            x.ma = Ka + Sa / x.W;
            x.mb = Kb + Sb / x.W;
            x.Maa = Saa - Sa * (Sa / x.W);
            x.Mbb = Sbb - Sb * (Sb / x.W);
            x.Mab = Sab - Sa * (Sb / x.W);
            m = merge(m, x);
        }
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) m = merge(m, shfl_moments(m, off));
        if (lane == 0) {
            const double va = m.Maa, vb = m.Mbb;
            double r = 0.0;
            if (va > 0.0 && vb > 0.0 && isfinite(va) && isfinite(vb)) r = m.Mab / sqrt(va * vb);
            fitness[p] = static_cast<float>(fabs(r));
            if (stats) {
                double* o = stats + p * kStats;
                o[0] = m.W; o[1] = m.ma; o[2] = m.mb; o[3] = m.Maa; o[4] = m.Mbb; o[5] = m.Mab;
                o[6] = r; o[7] = 0.0;
            }
        }
    } else {
        double s = 0.0, sw = 0.0;
        for (int c = lane; c < n_chunks; c += kWave) {
            s += part[p * n_chunks + c];
            if (has_w) sw += ystat[static_cast<int64_t>(c) * 4];
        }
        s = wave_sum(s);
        sw = has_w ? wave_sum(sw) : static_cast<double>(N);
        if (lane == 0) {
            double v = s / sw;
            if constexpr (METRIC == GP_METRIC_RMSE) v = sqrt(v);
            fitness[p] = static_cast<float>(v);
            if (stats) {
                double* o = stats + p * kStats;
                o[0] = sw; o[1] = o[2] = o[3] = o[4] = o[5] = 0.0; o[6] = v; o[7] = 0.0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_adjoint: derivative of every program's fitness with respect to each of
// its constants (not in the paper), by reverse mode over the compiled
// instructions, one wavefront per (row chunk, program) work item.
//
// Per tile of 64*R rows: a forward pass runs the stack machine and records
// on a tape the local derivatives each instruction will need (both partials
// of a product or quotient; the derivative of log, sqrt, sin, cos, tan at
// its input); the seed is d fitness / d yhat of each row; a reverse pass
// walks the instructions back with an adjoint stack that mirrors the value
// stack, multiplying by the taped partials, and at each constant reduces its
// adjoint over the wavefront into a per-program float64 sum.  Only
// instructions whose subtree holds a constant (kActive) record partials, and
// the reverse pass jumps over every subtree without one.  The first
// tape_lds_bytes<R>() of each wavefront's tape live in LDS, the rest (long
// programs) in a per-wavefront global area; the forward values are
// recomputed per tile, never kept.  Local derivatives (reading): add (1,1),
// sub (1,-1), mul (b,a), div (1/b, -a/b^2) if |b| > 0.001 else (0,0),
// log 1/a if |a| > 0.001 else 0, sqrt sign(a)/(2 sqrt|a|) (0 at a = 0),
// sin cos a, cos -sin a, tan 1 + tan^2 a, neg -1.
// ---------------------------------------------------------------------------
constexpr int kGradLds = 16;            // constants per program summed in a fixed order
// per-wavefront tape held in LDS: 12 KB, 15 KB at 4 rows per lane (two
// waves per SIMD there, so eight per CU still fit in LDS beside the 4 KB of
// function tables each holds)
template <int R>
constexpr int tape_lds_bytes() { return R == 4 ? 15360 : 12288; }

// tape entries an instruction records (0, 1 or 2)
__device__ __forceinline__ int tape_entries(uint32_t cls, uint32_t fn) {
    if (cls == kPush) return 0;
    if (cls == kUn) return fn == 0 ? 0 : 1;           // neg: the constant -1
    return fn >= 2 ? 2 : 0;                           // mul / div: both partials
}

// floats of a wavefront's global area: value- and adjoint-stack overflow, then
// the tape entries beyond those in LDS
template <int R>
constexpr int64_t adjoint_wave_floats(int64_t tape_entries_max) {
    const int64_t lds_entries = tape_lds_bytes<R>() / (R * kWave * 4);
    const int64_t beyond = tape_entries_max > lds_entries ? tape_entries_max - lds_entries : 0;
    return (2 * kStackLds + beyond) * R * kWave;
}

// derivative of unary function fn (1..5: log, sqrt, sin, cos, tan; 6..13:
// abs, exp, inv, sq, cube, tanh, atan, cbrt) at input x, whose result is y.
// Reciprocals here (and in the quotient's partials) come from the hardware
// reciprocal, within 1 ulp: a partial's own rounding, well inside the
// derivative tolerance, at a tenth of a correctly rounded division's cost.
// Every argument is normal: |x| > 0.001, 2 sqrt|x| >= 2^-73.5, 1 + x^2 >= 1,
// 3 cbrt(x)^2 >= 2^-99 for nonzero float x.
template <int R>
__device__ __forceinline__ void unary_derivative(uint32_t fn, const float (&x)[R], const float (&y)[R],
                                                 float (&dv)[R]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        switch (fn) {
        case 1: dv[j] = fabsf(x[j]) > GP_PROTECT_EPS ? __builtin_amdgcn_rcpf(x[j]) : 0.0f; break;
        case 2: dv[j] = x[j] == 0.0f ? 0.0f : copysignf(__builtin_amdgcn_rcpf(2.0f * y[j]), x[j]); break;
        case 3: dv[j] = cosf(x[j]); break;
        case 4: dv[j] = -sinf(x[j]); break;
        case 5: dv[j] = 1.0f + y[j] * y[j]; break;
        case 6: dv[j] = x[j] > 0.0f ? 1.0f : (x[j] < 0.0f ? -1.0f : 0.0f); break;
        case 7: dv[j] = y[j]; break;
        case 8: dv[j] = fabsf(x[j]) > GP_PROTECT_EPS ? -y[j] * y[j] : 0.0f; break;
        case 9: dv[j] = 2.0f * x[j]; break;
        case 10: dv[j] = 3.0f * (x[j] * x[j]); break;
        case 11: dv[j] = 1.0f - y[j] * y[j]; break;
        case 12: dv[j] = __builtin_amdgcn_rcpf(1.0f + x[j] * x[j]); break;
        default: dv[j] = y[j] != 0.0f ? __builtin_amdgcn_rcpf(3.0f * (y[j] * y[j])) : 0.0f; break;
        }
    }
}

template <int R, int FREG, int METRIC>
__global__ __launch_bounds__(kWave) void k_adjoint(PopView pop, CodeView cv, DataView d, Sched s,
                                                    const double* __restrict__ stats,
                                                    const double* __restrict__ wsum,
                                                    const float* __restrict__ gscale,
                                                    double* __restrict__ part,
                                                    double* __restrict__ gpart,
                                                    double* __restrict__ gextra,
                                                    float* __restrict__ gmem,
                                                    int64_t wave_floats) {
    constexpr int FA = FREG > 0 ? FREG : 1;
    constexpr int kTapeLds = tape_lds_bytes<R>() / (R * kWave * 4);
    const int lane = threadIdx.x;
    const int64_t N = d.N;
    const int64_t ld = d.ld;
    const float* __restrict__ X = d.X;
    __shared__ float ltape[kTapeLds * R * kWave];
    __shared__ double gw[kGradLds];
    float* __restrict__ wmem = gmem + static_cast<int64_t>(blockIdx.x) * wave_floats;
    float* __restrict__ ovf = wmem;                                 // value stack beyond registers
    float* __restrict__ aovf = wmem + kStackLds * R * kWave;        // adjoint stack beyond registers
    float* __restrict__ gtape = wmem + 2 * kStackLds * R * kWave;   // tape entries beyond LDS
    const double W = *wsum;
    // (the function tables' LDS copy takes the 4 KB the tape gives up at
    // four rows per lane: eight wavefronts per CU still fit)
    __shared__ MathTabsLds tabs_lds;
    const MathTabs mt = stage_tabs(tabs_lds);

    // entry e of row slot j: LDS for e < kTapeLds, the global area beyond
    auto tape_put = [&](int e, const float (&v)[R]) {
        if (e < kTapeLds) {
#pragma unroll
            for (int j = 0; j < R; ++j) ltape[(e * R + j) * kWave + lane] = v[j];
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) gtape[((e - kTapeLds) * R + j) * kWave + lane] = v[j];
        }
    };
    auto tape_get = [&](int e, float (&v)[R]) {
        if (e < kTapeLds) {
#pragma unroll
            for (int j = 0; j < R; ++j) v[j] = ltape[(e * R + j) * kWave + lane];
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) v[j] = gtape[((e - kTapeLds) * R + j) * kWave + lane];
        }
    };

    // work items: the evaluation kernel's per-XCD queues, one item per claim
    const int q0 = static_cast<int>(blockIdx.x % kQueues);
    int qi = 0;
    for (;;) {
        int64_t it = -1;
        int qx = q0;
        while (qi < kQueues) {
            qx = (q0 + qi) % kQueues;
            const int64_t q_items = (static_cast<int64_t>(s.n_chunks) - qx + kQueues - 1) / kQueues * pop.P;
            uint32_t it32 = 0;
            if (lane == 0) it32 = atomicAdd(s.counter + qx * kQueueStride, 1u);
            const int64_t cand = static_cast<int64_t>(
                static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(it32), 0)));
            if (cand < q_items) {
                it = cand;
                break;
            }
            ++qi;   // this queue is dry
        }
        if (it < 0) break;   // every queue is dry
        const int32_t cq = static_cast<int32_t>(it / pop.P);
        const int32_t k = static_cast<int32_t>(it - static_cast<int64_t>(cq) * pop.P);
        const int32_t c = cq * kQueues + qx;
        const int32_t p = ldu(s.order + k);
        const int64_t off = ldu(pop.prog_off + p);
        const int32_t CL = ldu(cv.clen + p);
        const int64_t cbase = ldu(pop.const_off + p);
        const int32_t nconst = static_cast<int32_t>(ldu(pop.const_off + p + 1) - cbase);
        const uint4* __restrict__ pcode = cv.code + off;
        const int64_t r0 = static_cast<int64_t>(c) * s.chunk;
        const int64_t r1 = min(r0 + s.chunk, N);
        const float gsc = gscale ? ldu(gscale + p) : 1.0f;
        double sm0 = 0.0, sm1 = 0.0, sm2 = 0.0, sm3 = 0.0, sm4 = 0.0, sm5 = 0.0, sm6 = 0.0;
        if (stats) {
            sm0 = stats[p * kStats + 0]; sm1 = stats[p * kStats + 1]; sm2 = stats[p * kStats + 2];
            sm3 = stats[p * kStats + 3]; sm4 = stats[p * kStats + 4]; sm5 = stats[p * kStats + 5];
            sm6 = stats[p * kStats + 6];
        }
        (void)sm0; (void)sm5;
        const int nlds = min(nconst, kGradLds);
        if (lane < nlds) gw[lane] = 0.0;
        __syncthreads();
        double lacc = 0.0;
        // a program without constants needs only its loss, and only when asked
        const int64_t r_end = (nconst == 0 && !part) ? r0 : r1;

        for (int64_t base = r0; base < r_end; base += kWave * R) {
            int64_t row[R];
            bool valid[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int64_t r = base + j * kWave + lane;
                valid[j] = r < r1;
                row[j] = valid[j] ? r : r1 - 1;
            }
            GP_ARRAYS(xa, FA);
            if constexpr (FREG > 0) {
#pragma unroll
                for (int f = 0; f < FREG; ++f) {
                    if (f < d.F) {
                        xa0[f] = X[f * ld + row[0]];
                        if constexpr (R > 1) xa1[f] = X[f * ld + row[1]];
                        if constexpr (R > 2) xa2[f] = X[f * ld + row[2]];
                        if constexpr (R > 3) xa3[f] = X[f * ld + row[3]];
                    }
                }
            }
            // ---------------- forward pass, recording the tape ----------------
            float t[R];
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = 0.0f;
            GP_ARRAYS(st, kStackRegs + 1);
            int dp = -1;
            int ntape = 0;
            uint4 nxt = pcode[0];
            for (int q = 0; q < CL; ++q) {
                const uint4 cur = nxt;
                nxt = pcode[min(q + 1, CL - 1)];
                const uint32_t w = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.x)));
                const uint32_t cls = w & 3u;
                const uint32_t fn = (w >> 2) & 15u;
                const bool act = (w & kActive) != 0u;
                GP_PUT(st, min(dp + 1, kStackRegs), t);
                float a[R], b[R];
                bool binary = false;
                if (cls == kUn) {
                    float x[R];
#pragma unroll
                    for (int j = 0; j < R; ++j) x[j] = t[j];
                    apply_unary<R, true>(fn, t, mt);
                    if (fn != 0 && act) {
                        float dv[R];
                        unary_derivative<R>(fn, x, t, dv);
                        tape_put(ntape, dv);
                        ++ntape;
                    }
                } else if (cls == kBin) {
                    if (dp < kStackRegs) {
                        GP_GET(st, dp, b);
                    } else {
#pragma unroll
                        for (int j = 0; j < R; ++j) b[j] = ovf[((dp - kStackRegs) * R + j) * kWave + lane];
                    }
                    --dp;
#pragma unroll
                    for (int j = 0; j < R; ++j) a[j] = t[j];
                    binary = true;
                } else {
                    float v[R];
                    if (w & kConstBit) {
                        const float cval = __uint_as_float(cur.y);
#pragma unroll
                        for (int j = 0; j < R; ++j) v[j] = cval;
                    } else if constexpr (FREG > 0) {
                        const uint32_t arg = w >> 8;
                        v[0] = xa0[arg];
                        if constexpr (R > 1) v[1] = xa1[arg];
                        if constexpr (R > 2) v[2] = xa2[arg];
                        if constexpr (R > 3) v[3] = xa3[arg];
                    } else {
                        const float* __restrict__ col = X + static_cast<int64_t>(w >> 8) * ld;
#pragma unroll
                        for (int j = 0; j < R; ++j) v[j] = col[row[j]];
                    }
                    if (cls == kPush) {
                        ++dp;
                        if (dp >= kStackRegs) {
#pragma unroll
                            for (int j = 0; j < R; ++j) ovf[((dp - kStackRegs) * R + j) * kWave + lane] = t[j];
                        }
#pragma unroll
                        for (int j = 0; j < R; ++j) t[j] = v[j];
                    } else {
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            a[j] = v[j];
                            b[j] = t[j];
                        }
                        binary = true;
                    }
                }
                if (binary) {
                    if (fn >= 2 && act) {   // mul, div, max, min, atan2: both partials
                        float da[R], db[R];
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            if (fn == 2) {
                                da[j] = b[j];
                                db[j] = a[j];
                            } else if (fn == 3) {
                                if (fabsf(b[j]) > GP_PROTECT_EPS) {
                                    const float inv = __builtin_amdgcn_rcpf(b[j]);
                                    da[j] = inv;
                                    db[j] = -a[j] * inv * inv;
                                } else {
                                    da[j] = 0.0f;
                                    db[j] = 0.0f;
                                }
                            } else if (fn == 4 || fn == 5) {
                                // the selected operand (the first on ties) carries it
                                const bool first = (fn == 4 ? a[j] >= b[j] : a[j] <= b[j]) || isnan(b[j]);
                                da[j] = first ? 1.0f : 0.0f;
                                db[j] = first ? 0.0f : 1.0f;
                            } else {
                                const float r2 = a[j] * a[j] + b[j] * b[j];
                                da[j] = r2 > 0.0f ? b[j] / r2 : 0.0f;
                                db[j] = r2 > 0.0f ? -a[j] / r2 : 0.0f;
                            }
                        }
                        tape_put(ntape, da);
                        tape_put(ntape + 1, db);
                        ntape += 2;
                    }
                    apply_binary<R>(fn, a, b);
#pragma unroll
                    for (int j = 0; j < R; ++j) t[j] = a[j];
                }
                // the chained unary functions, each taping its derivative
                for (uint32_t ch = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.z)));
                     ch != 0u; ch >>= 4) {
                    const uint32_t u = (ch & 15u) - 1u;
                    float x[R];
#pragma unroll
                    for (int j = 0; j < R; ++j) x[j] = t[j];
                    apply_unary<R, true>(u, t, mt);
                    if (u != 0 && act) {
                        float dv[R];
                        unary_derivative<R>(u, x, t, dv);
                        tape_put(ntape, dv);
                        ++ntape;
                    }
                }
            }

            // ---------------- seeds: d fitness / d yhat per row ----------------
            float g[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const double yh = static_cast<double>(t[j]);
                const double yv = static_cast<double>(d.y[row[j]]);
                const double wv = d.w ? static_cast<double>(d.w[row[j]]) : 1.0;
                double sd;
                if constexpr (METRIC == GP_METRIC_MSE) {
                    const double e = yh - yv;
                    sd = 2.0 * wv * e / W;
                    lacc += valid[j] ? wv * (e * e) : 0.0;
                } else if constexpr (METRIC == GP_METRIC_RMSE) {
                    const double e = yh - yv;
                    sd = sm6 > 0.0 ? (wv * e / W) / sm6 : 0.0;
                } else if constexpr (METRIC == GP_METRIC_MAE) {
                    const double e = yh - yv;
                    sd = wv * (e > 0.0 ? 1.0 : (e < 0.0 ? -1.0 : 0.0)) / W;
                    lacc += valid[j] ? wv * fabs(e) : 0.0;
                } else if constexpr (METRIC == GP_METRIC_LOGLOSS) {
                    const float z = t[j];
                    const float yf = d.y[row[j]];
                    const float t1 = fmaxf(z, 0.0f);
                    const float t2 = yf * z;
                    const float t3 = t1 - t2;
                    const float t5 = log1pf(expf(-fabsf(z)));
                    lacc += valid[j] ? wv * static_cast<double>(t3 + t5) : 0.0;
                    sd = wv * (1.0 / (1.0 + exp(-yh)) - yv) / W;
                } else {  // PEARSON: d|r|/dyhat
                    const double va = sm3, vb = sm4, rr = sm6;
                    if (va > 0.0 && vb > 0.0 && isfinite(va) && isfinite(vb)) {
                        const double dr = wv * ((yv - sm2) / sqrt(va * vb) - rr * (yh - sm1) / va);
                        sd = rr >= 0.0 ? dr : -dr;
                    } else {
                        sd = 0.0;
                    }
                }
                g[j] = valid[j] ? static_cast<float>(sd) * gsc : 0.0f;
            }

            if (nconst == 0) continue;   // no constant: nothing to carry back
            // ---------------- reverse pass ----------------
            GP_ARRAYS(as, kStackRegs + 1);   // adjoints of the entries below the top
            int ad = dp;                     // mirrors the value stack (dp == 0 here)
            // the walk visits the active instructions through their links (the
            // root, the last instruction, is active: the program holds a
            // constant); the next one is fetched while this one runs
            uint4 cur = pcode[CL - 1];
            for (;;) {
                const uint32_t link = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.w)));
                const int qn = static_cast<int>(link & kNextMask) - 1;
                const uint4 nxt_ins = pcode[max(qn, 0)];
                const uint32_t w = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.x)));
                const uint32_t cls = w & 3u;
                const uint32_t fn = (w >> 2) & 15u;
                // the chained unary functions first, the last one first
                const uint32_t chain = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.z)));
                if (chain != 0u) {
                    const int nch = (32 - __clz(static_cast<int>(chain)) + 3) >> 2;
                    for (int kq = nch - 1; kq >= 0; --kq) {
                        const uint32_t u = ((chain >> (4 * kq)) & 15u) - 1u;
                        if (u == 0u) {
#pragma unroll
                            for (int j = 0; j < R; ++j) g[j] = -g[j];
                        } else {
                            --ntape;
                            float dv[R];
                            tape_get(ntape, dv);
#pragma unroll
                            for (int j = 0; j < R; ++j) g[j] = g[j] * dv[j];
                        }
                    }
                }
                const int ne = tape_entries(cls, fn);
                ntape -= ne;
                float gb[R];   // adjoint handed to the entry below the top (binary only)
#pragma unroll
                for (int j = 0; j < R; ++j) gb[j] = 0.0f;
                float gc[R];   // adjoint of the terminal (push / fold)
#pragma unroll
                for (int j = 0; j < R; ++j) gc[j] = 0.0f;
                if (cls == kUn) {
                    if (ne == 0) {
#pragma unroll
                        for (int j = 0; j < R; ++j) g[j] = -g[j];
                    } else {
                        float dv[R];
                        tape_get(ntape, dv);
#pragma unroll
                        for (int j = 0; j < R; ++j) g[j] = g[j] * dv[j];
                    }
                } else if (cls == kPush) {
#pragma unroll
                    for (int j = 0; j < R; ++j) gc[j] = g[j];
                } else {
                    // binary: operands (a, b); fold: a is the terminal, b the old top
                    float ga[R];
                    if (ne == 0) {
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            ga[j] = g[j];
                            gb[j] = fn == 0 ? g[j] : -g[j];
                        }
                    } else {
                        float da[R], db[R];
                        tape_get(ntape, da);
                        tape_get(ntape + 1, db);
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            ga[j] = g[j] * da[j];
                            gb[j] = g[j] * db[j];
                        }
                    }
                    if (cls == kBin) {
#pragma unroll
                        for (int j = 0; j < R; ++j) g[j] = ga[j];
                    } else {
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            gc[j] = ga[j];
                            g[j] = gb[j];
                        }
                    }
                }
                // adjoint stack: a binary hands gb to the (restored) entry below
                GP_PUT(as, min(ad + 1, kStackRegs), gb);
                if (cls == kBin) {
                    ++ad;
                    if (ad >= kStackRegs) {
#pragma unroll
                        for (int j = 0; j < R; ++j) aovf[((ad - kStackRegs) * R + j) * kWave + lane] = gb[j];
                    }
                }
                // a constant terminal: its adjoint summed over the wavefront's rows
                if (cls <= kFold && (w & kConstBit)) {
                    const int slot = static_cast<int>(w >> 8);
                    double sum = 0.0;
#pragma unroll
                    for (int j = 0; j < R; ++j) sum += valid[j] ? static_cast<double>(gc[j]) : 0.0;
                    const double tot = wave_sum(sum);
                    if (lane == 0) {
                        if (slot < kGradLds) gw[slot] += tot;
                        else atomicAdd(gextra + cbase + slot, tot);
                    }
                }
                // a push is undone, and so is each skipped subtree (one value on
                // the stack, carrying nothing back): the entry below becomes
                // the top again
                const int undo = (cls == kPush ? 1 : 0) + static_cast<int>(link >> kNextBits);
                if (undo > 0) {
                    ad -= undo;
                    const int top = ad + 1;
                    if (top >= 0) {
                        if (top < kStackRegs) {
                            GP_GET(as, top, g);
                        } else {
#pragma unroll
                            for (int j = 0; j < R; ++j) g[j] = aovf[((top - kStackRegs) * R + j) * kWave + lane];
                        }
                    }
                }
                if (qn < 0) break;
                cur = nxt_ins;
            }
        }
        // ---------------- per-item results ----------------
        __syncthreads();
        if (lane < nlds) gpart[(cbase + lane) * s.n_chunks + c] = gw[lane];
        if (part) {
            lacc = wave_sum(lacc);
            if (lane == 0) part[static_cast<int64_t>(p) * s.n_chunks + c] = lacc;
        }
        __syncthreads();
    }
}

// grad[i] = sum over chunks of gpart[i * n_chunks + c] (fixed order) plus
// gextra[i]; one lane per constant.
__global__ __launch_bounds__(kBlock) void k_finalize_grad(const double* __restrict__ gpart,
                                                           const double* __restrict__ gextra,
                                                           const int64_t* __restrict__ const_off,
                                                           int32_t P, int32_t n_chunks,
                                                           float* __restrict__ grad) {
    const int32_t p = static_cast<int32_t>(blockIdx.x) * (kBlock / kWave) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    if (p >= P) return;
    const int64_t c0 = const_off[p], c1 = const_off[p + 1];
    for (int64_t i = c0 + lane; i < c1; i += kWave) {
        double sum = gextra[i];
        if (i - c0 < kGradLds)
            for (int c = 0; c < n_chunks; ++c) sum += gpart[i * n_chunks + c];
        grad[i] = static_cast<float>(sum);
    }
}

__global__ __launch_bounds__(kBlock) void k_zero(double* __restrict__ p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// sum of weights over all rows (float64), from the per-chunk statistics
__global__ __launch_bounds__(kWave) void k_wsum(const double* __restrict__ ystat, int32_t n_chunks,
                                                 int has_w, int64_t N, double* __restrict__ out) {
    double s = 0.0;
    if (has_w)
        for (int c = threadIdx.x; c < n_chunks; c += kWave) s += ystat[static_cast<int64_t>(c) * 4];
    s = wave_sum(s);
    if (threadIdx.x == 0) *out = has_w ? s : static_cast<double>(N);
}

// ---------------------------------------------------------------------------
// k_tournament (Sec. III-C1): one lane per tournament.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_tournament(const float* __restrict__ fit,
                                                        const int32_t* __restrict__ len,
                                                        int32_t P, int larger, float c, int32_t k,
                                                        int32_t T, uint64_t seed, uint32_t gen_value,
                                                        const uint32_t* __restrict__ gen_dev,
                                                        int32_t* __restrict__ winners) {
    const int32_t t = static_cast<int32_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= T) return;
    // a captured generation graph reads the generation number from memory
    const uint32_t gen = gen_dev ? *gen_dev : gen_value;
    int32_t best = -1;
    float best_adj = 0.0f;
    Philox4 blk{};
    for (int32_t dd = 0; dd < k; ++dd) {
        if ((dd & 3) == 0) blk = philox4x32_10(static_cast<uint32_t>(dd >> 2), static_cast<uint32_t>(t), gen,
                                               kStreamTournament, seed);
        const int32_t idx = static_cast<int32_t>(below(blk.v[dd & 3], static_cast<uint32_t>(P)));
        const float pen = __fmul_rn(c, static_cast<float>(len[idx]));
        const float raw = fit[idx];
        const float adj = larger ? __fsub_rn(raw, pen) : __fadd_rn(raw, pen);
        bool take;
        if (best < 0) take = true;
        else if (isnan(adj)) take = false;
        else if (isnan(best_adj)) take = true;
        else take = larger ? (adj > best_adj) : (adj < best_adj);
        if (take) {
            best = idx;
            best_adj = adj;
        }
    }
    winners[t] = best;
}

// ---------------------------------------------------------------------------
// Spearman (Sec. III-C3 ranks each program's outputs with a sort): the outputs
// of a batch of programs become order-preserving 32-bit keys in the first
// pass of a segmented LSD radix sort (four passes of 8 bits: per-tile digit
// counts, a per-segment scan, a stable scatter), each carrying its row's
// target rank (or its row, with weights) through the sort, and one workgroup
// per program walks its sorted keys, giving tied values the mean of their
// ranks, and forms the float64 moments of the (value rank, target rank)
// pairs.
// ---------------------------------------------------------------------------
constexpr int kRsBlock = 256;                  // threads of the count kernel
constexpr int kRsScatterBlock = 512;           // threads of the scatter
constexpr int kRsItems = 16;                   // keys per scatter thread
constexpr int kRsTile = kRsScatterBlock * kRsItems;   // keys per tile
constexpr int kRsRadix = 256;

// float -> uint32 with the same order; -0 and +0 map to one key
__device__ __forceinline__ uint32_t order_key(float v) {
    uint32_t b = __float_as_uint(v == 0.0f ? 0.0f : v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// counts[(seg * 256 + digit) * T + tile] for one pass.  The first pass reads
// the float values themselves (their order-preserving keys are formed here)
// and raises nan[seg] for a NaN.
template <bool FIRST>
__global__ __launch_bounds__(kRsBlock) void k_rs_count(const uint32_t* __restrict__ keys, int64_t N, int32_t T,
                                                        int shift, uint32_t* __restrict__ counts,
                                                        int32_t* __restrict__ nan_flag) {
    __shared__ uint32_t hist[kRsRadix];
    const int32_t tile = blockIdx.x, seg = blockIdx.y;
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(seg) * N;
    const int64_t t0 = static_cast<int64_t>(tile) * kRsTile;
    for (int k = 0; k < kRsTile / kRsBlock; ++k) {
        const int64_t i = t0 + k * kRsBlock + threadIdx.x;
        if (i < N) {
            uint32_t key = keys[base + i];
            if constexpr (FIRST) {
                const float v = __uint_as_float(key);
                if (isnan(v)) nan_flag[seg] = 1;
                key = order_key(v);
            }
            atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    counts[(static_cast<int64_t>(seg) * kRsRadix + threadIdx.x) * T + tile] = hist[threadIdx.x];
}

// exclusive scan of one segment's 256*T counts, digit-major (in place), in
// chunks of 1,024 consecutive counts (coalesced; four chunks' loads issued
// together): shuffle scans within each wavefront, the wavefronts' totals
// through LDS (double-buffered, so one barrier per chunk), then the carry of
// the earlier chunks.
__global__ __launch_bounds__(1024) void k_rs_scan(uint32_t* __restrict__ counts, int32_t T) {
    constexpr int kW = 1024 / kWave, kE = 4;
    __shared__ uint32_t wtot[2][kW];
    const int64_t n = static_cast<int64_t>(kRsRadix) * T;
    uint32_t* c = counts + static_cast<int64_t>(blockIdx.x) * n;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid >> 6;
    uint32_t carry = 0;
    int par = 0;
    for (int64_t c0 = 0; c0 < n; c0 += 1024 * kE) {
        uint32_t v[kE];
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const int64_t i = c0 + e * 1024 + tid;
            v[e] = i < n ? c[i] : 0u;
        }
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            uint32_t x = v[e];
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t o = __shfl_up(x, d, kWave);
                if (lane >= d) x += o;
            }
            if (lane == kWave - 1) wtot[par][wid] = x;
            __syncthreads();
            uint32_t pre = carry, all = carry;
            for (int q = 0; q < kW; ++q) {
                const uint32_t t = wtot[par][q];
                pre += q < wid ? t : 0u;
                all += t;
            }
            const int64_t i = c0 + e * 1024 + tid;
            if (i < n) c[i] = pre + x - v[e];
            carry = all;
            par ^= 1;
        }
    }
}

// stable scatter of one tile, staged through LDS.  Wavefront w takes the
// tile's keys w*1024 ... w*1024+1023 in index order, 64 a round; within a
// round, lanes holding the same digit find each other by ballots over the
// digit's bits, and the wavefront's running count of that digit (its own row
// of LDS counters, updated by the lowest such lane; a wavefront's LDS
// operations are ordered, so no barrier is needed) gives each key its rank
// among the wavefront's keys of that digit.  One barrier later, each digit's
// counts are turned into exclusive prefixes over the wavefronts, which puts
// every key at its digit-sorted position within the tile in LDS.  The tile
// then goes out run by run: consecutive threads write consecutive addresses
// of each digit's output range.  The tile's count of digit d is the
// difference of adjacent scanned offsets (digit-major over tiles, the last
// one closed by N).  The first pass reads the float values, forms their
// keys, and gives each the value it carries through the sort: its row's
// target rank where rank2_y is given (then the sorted values are the target
// ranks in the program's order), else its row.
template <bool FIRST>
__global__ __launch_bounds__(kRsScatterBlock) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          int64_t N, int32_t T, int shift,
                                                          const uint32_t* __restrict__ offsets,
                                                          const uint32_t* __restrict__ rank2_y) {
    constexpr int kWaves = kRsScatterBlock / kWave;
    constexpr int kDigitWaves = kRsRadix / kWave;     // the wavefronts that keep one digit per thread
    constexpr int kPerWave = kRsTile / kWaves;        // keys per wavefront (kRsItems rounds of 64)
    __shared__ uint32_t base_off[kRsRadix];           // global start of each digit for this tile
    __shared__ uint32_t loc_off[kRsRadix];            // local start of each digit within the tile
    __shared__ uint32_t hist[kWaves][kRsRadix];       // per-wavefront digit counts, then their prefixes
    __shared__ uint32_t wsum[kDigitWaves];
    __shared__ uint32_t skey[kRsTile], sval[kRsTile];
    const int32_t tile = blockIdx.x, seg = blockIdx.y;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    // threads below kRsRadix keep digit tid's offsets
    const bool digit_thread = tid < kRsRadix;
    uint32_t start = 0, cnt = 0;
    if (digit_thread) {
        const int64_t cidx = (static_cast<int64_t>(seg) * kRsRadix + tid) * T + tile;
        const int64_t nidx = static_cast<int64_t>(kRsRadix) * T;     // offsets per segment
        start = offsets[cidx];
        const int64_t cnext = (static_cast<int64_t>(tid) * T + tile + 1 < nidx) ? cidx + 1 : -1;
        cnt = (cnext >= 0 ? offsets[cnext] : static_cast<uint32_t>(N)) - start;
    }
    const int64_t sbase = static_cast<int64_t>(seg) * N;
    const int64_t t0 = static_cast<int64_t>(tile) * kRsTile;
    const int tile_len = static_cast<int>(min<int64_t>(kRsTile, N - t0));
    // this wavefront's keys, all loads issued before the ranking
    uint32_t pkey[kRsItems], pval[kRsItems];
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t i = t0 + wave * kPerWave + k * kWave + lane;
        if constexpr (FIRST) {
            pkey[k] = i < N ? order_key(__uint_as_float(kin[sbase + i])) : 0u;
            pval[k] = i < N ? (rank2_y ? rank2_y[i] : static_cast<uint32_t>(i)) : 0u;
        } else {
            pkey[k] = i < N ? kin[sbase + i] : 0u;
            pval[k] = i < N ? vin[sbase + i] : 0u;
        }
    }
    if (digit_thread) {
        base_off[tid] = start;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) hist[w][tid] = 0;
    }
    // exclusive scan of the tile's digit counts (shuffles within each wave,
    // then the waves' totals)
    uint32_t v = cnt;
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    if (digit_thread && lane == kWave - 1) wsum[wave] = v;
    __syncthreads();
    if (digit_thread) {
        uint32_t pre = 0;
        for (int q = 0; q < wave; ++q) pre += wsum[q];
        loc_off[tid] = pre + v - cnt;
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t prank[kRsItems];
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t i = t0 + wave * kPerWave + k * kWave + lane;
        const bool valid = i < N;
        const uint32_t d = (pkey[k] >> shift) & 255u;
        // lanes of this wave holding a valid key with the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bal = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bal : ~bal;
        }
        const uint32_t rank_w = static_cast<uint32_t>(__popcll(peers & lt_mask));
        const uint32_t before = hist[wave][d];
        prank[k] = before + rank_w;
        if (valid && rank_w == 0) hist[wave][d] = before + static_cast<uint32_t>(__popcll(peers));
    }
    __syncthreads();
    if (digit_thread) {   // exclusive prefix over the wavefronts of digit tid's counts
        uint32_t acc = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = hist[w][tid];
            hist[w][tid] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t i = t0 + wave * kPerWave + k * kWave + lane;
        if (i < N) {
            const uint32_t d = (pkey[k] >> shift) & 255u;
            const uint32_t lp = loc_off[d] + hist[wave][d] + prank[k];
            if (lp < static_cast<uint32_t>(kRsTile)) {
                skey[lp] = pkey[k];
                sval[lp] = pval[k];
            }
        }
    }
    __syncthreads();
    // the tile, digit-sorted, to its digits' output ranges
    for (int j = tid; j < tile_len; j += kRsScatterBlock) {
        const uint32_t key = skey[j];
        const uint32_t d = (key >> shift) & 255u;
        const uint32_t pos = base_off[d] + (static_cast<uint32_t>(j) - loc_off[d]);
        if (pos < static_cast<uint64_t>(N)) {
            kout[sbase + pos] = key;
            vout[sbase + pos] = sval[j];
        }
    }
}

// The target's ranks, from its sorted keys (one workgroup): rank2[row] is
// twice the mean rank of the tied run holding the row, an integer.  Pass A,
// ascending chunks of 1,024: the start of the run holding position i (an
// inclusive max-scan: shuffles within each wavefront, the wavefronts' totals
// through LDS, the carry of earlier chunks), kept in run_start.  Pass B,
// descending: the end of the run (the mirror min-scan from the right), and
// the weighted sums (w, w b, w b^2) of the centred ranks b = rank - (N+1)/2,
// which every program's correlation shares (tsum).
__global__ __launch_bounds__(1024) void k_spear_rank_target(const uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ idx, int64_t N,
                                                             const float* __restrict__ w,
                                                             uint32_t* __restrict__ run_start,
                                                             uint32_t* __restrict__ rank2_out,
                                                             double* __restrict__ tsum) {
    constexpr int kW = 1024 / kWave;                 // wavefronts in the block
    __shared__ uint32_t wtot[kW];
    __shared__ double red[3][kW];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wid = tid >> 6;
    const uint32_t* k = keys;
    uint32_t* rs = run_start;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < N; c0 += 1024) {
        const int64_t i = c0 + tid;
        uint32_t v = 0;
        if (i < N) v = (i == 0 || k[i] != k[i - 1]) ? static_cast<uint32_t>(i) : 0u;
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_up(v, d, kWave);
            if (lane >= d) v = max(v, o);
        }
        if (lane == kWave - 1) wtot[wid] = v;
        __syncthreads();
        uint32_t pre = carry, all = carry;
        for (int q = 0; q < kW; ++q) {
            const uint32_t t = wtot[q];
            if (q < wid) pre = max(pre, t);
            all = max(all, t);
        }
        if (i < N) rs[i] = max(v, pre);
        __syncthreads();
        carry = all;
    }
    const double mid = 0.5 * (static_cast<double>(N) + 1.0);
    double s_w = 0.0, s_b = 0.0, s_bb = 0.0;
    uint32_t carry_end = static_cast<uint32_t>(N);
    for (int64_t c1 = ((N + 1023) / 1024) * 1024; c1 > 0; c1 -= 1024) {
        const int64_t i = c1 - 1024 + tid;
        uint32_t v = 0xffffffffu;
        if (i < N) v = (i == N - 1 || k[i] != k[i + 1]) ? static_cast<uint32_t>(i + 1) : 0xffffffffu;
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_down(v, d, kWave);
            if (lane + d < kWave) v = min(v, o);
        }
        if (lane == 0) wtot[wid] = v;
        __syncthreads();
        uint32_t suf = carry_end, all = carry_end;
        for (int q = 0; q < kW; ++q) {
            const uint32_t t = wtot[q];
            if (q > wid) suf = min(suf, t);
            all = min(all, t);
        }
        if (i < N) {
            const uint32_t row = idx[i];
            const uint32_t r2 = rs[i] + 1u + min(v, suf);
            rank2_out[row] = r2;
            const double wv = w ? static_cast<double>(w[row]) : 1.0;
            const double b = 0.5 * static_cast<double>(r2) - mid;
            s_w += wv;
            s_b += wv * b;
            s_bb += wv * b * b;
        }
        __syncthreads();
        carry_end = all;
    }
    double v[3] = {s_w, s_b, s_bb};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double t = wave_sum(v[q]);
        if (lane == 0) red[q][wid] = t;
    }
    __syncthreads();
    if (tid < 3) {
        double acc = 0.0;
        for (int j = 0; j < kW; ++j) acc += red[tid][j];
        tsum[tid] = acc;
    }
}

// Rank correlation of a batch of programs, one workgroup per program and one
// pass over its sorted keys.  The tied run holding position i spans
// [start, end) and twice its mean rank is start + 1 + end.  Each block of
// 1,024 positions finds starts by a max-scan from the left and ends by a
// min-scan from the right (wavefront shuffles, the wavefronts' totals in
// double-buffered LDS: one barrier per block of positions).  A run that
// reaches past the block is still open: each thread sums its rows' weights
// and weighted target ranks for it, and folds those sums in with the run's
// mean rank in the block whose first end closes the run (its start is then
// the carry of the earlier blocks).  With a = rank - (N+1)/2 for the program
// and b likewise for the target, the weighted sums of a, a^2 and a b and the
// target's shared sums (tsum) give |r|: 0 for a constant rank vector, NaN if
// the outputs or the target held a NaN.  Two blocks' loads go out together.
// Unweighted, the sorted values are the target ranks themselves; weighted,
// they are rows, whose target ranks and weights are gathered.
template <bool WEIGHTED>
__global__ __launch_bounds__(1024) void k_spear_corr(const uint32_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals, int64_t N,
                                                      const uint32_t* __restrict__ rank2_y,
                                                      const float* __restrict__ w,
                                                      const double* __restrict__ tsum,
                                                      const int32_t* __restrict__ nan_flag,
                                                      const int32_t* __restrict__ target_nan,
                                                      float* __restrict__ fitness, int32_t prog0) {
    constexpr int kW = 1024 / kWave, kE = 2;
    constexpr uint32_t kNone = 0xffffffffu;
    __shared__ uint32_t wmax[2][kW], wmin[2][kW];
    __shared__ double red[3][kW];
    const int32_t seg = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wid = tid >> 6;
    const uint32_t n = static_cast<uint32_t>(N);      // below 2^31
    const uint32_t* k = keys + static_cast<int64_t>(seg) * N;
    const uint32_t* ix = vals + static_cast<int64_t>(seg) * N;
    const double mid = 0.5 * (static_cast<double>(N) + 1.0);
    double s_a = 0.0, s_aa = 0.0, s_ab = 0.0;
    double o_w = 0.0, o_wb = 0.0;     // this thread's rows of the open run
    uint32_t carry = 0;               // start of the last run so far
    int par = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += 1024 * kE) {
        uint32_t kc[kE], ry[kE];
        float wf[kE];
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const uint32_t i = c0 + e * 1024 + tid;
            kc[e] = i < n ? k[i] : 0u;
            ry[e] = i < n ? ix[i] : 0u;
        }
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const uint32_t i = c0 + e * 1024 + tid;
            const uint32_t row = ry[e];
            if constexpr (WEIGHTED) {
                ry[e] = i < n ? rank2_y[row] : 0u;
                wf[e] = i < n ? w[row] : 1.0f;
            } else {
                wf[e] = 1.0f;
            }
        }
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const uint32_t i = c0 + e * 1024 + tid;
            const bool in = i < n;
            // neighbours by shuffles, loads at the wavefront's edges
            uint32_t kp = __shfl_up(kc[e], 1, kWave), kn = __shfl_down(kc[e], 1, kWave);
            if (lane == 0) kp = (in && i > 0) ? k[i - 1] : 0u;
            if (lane == kWave - 1) kn = (i + 1 < n) ? k[i + 1] : 0u;
            const bool start = in && (i == 0 || kc[e] != kp);
            const bool end = in && (i == n - 1 || kc[e] != kn);
            uint32_t vs = start ? i : 0u;
            uint32_t ve = end ? i + 1 : kNone;
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t os = __shfl_up(vs, d, kWave);
                const uint32_t oe = __shfl_down(ve, d, kWave);
                if (lane >= d) vs = max(vs, os);
                if (lane + d < kWave) ve = min(ve, oe);
            }
            if (lane == kWave - 1) wmax[par][wid] = vs;
            if (lane == 0) wmin[par][wid] = ve;
            __syncthreads();
            // the wavefronts' totals, lane q holding wavefront q's: a prefix
            // max and a suffix min over them by shuffles
            uint32_t tm = lane < kW ? wmax[par][lane] : 0u;
            uint32_t te = lane < kW ? wmin[par][lane] : kNone;
            for (int d = 1; d < kW; d <<= 1) {
                const uint32_t om = __shfl_up(tm, d, kWave);
                const uint32_t oe = __shfl_down(te, d, kWave);
                if (lane >= d) tm = max(tm, om);
                if (lane + d < kWave) te = min(te, oe);
            }
            const uint32_t pre = max(carry, wid > 0 ? static_cast<uint32_t>(__shfl(tm, wid - 1, kWave)) : 0u);
            const uint32_t all = max(carry, static_cast<uint32_t>(__shfl(tm, kW - 1, kWave)));
            const uint32_t suf = wid < kW - 1 ? static_cast<uint32_t>(__shfl(te, wid + 1, kWave)) : kNone;
            const uint32_t first_end = __shfl(te, 0, kWave);
            if (first_end != kNone) {       // the open run (if any) ends here
                const double a = 0.5 * (static_cast<double>(carry) + 1.0 + static_cast<double>(first_end)) - mid;
                s_a += a * o_w;
                s_aa += a * a * o_w;
                s_ab += a * o_wb;
                o_w = 0.0;
                o_wb = 0.0;
            }
            if (in) {
                const double wv = static_cast<double>(wf[e]);
                const double b = 0.5 * static_cast<double>(ry[e]) - mid;
                const uint32_t en = min(ve, suf);
                if (en != kNone) {
                    const double a = 0.5 * (static_cast<double>(max(vs, pre)) + 1.0 + static_cast<double>(en)) - mid;
                    s_a += wv * a;
                    s_aa += wv * a * a;
                    s_ab += wv * a * b;
                } else {
                    o_w += wv;
                    o_wb += wv * b;
                }
            }
            carry = all;
            par ^= 1;
        }
    }
    double v[3] = {s_a, s_aa, s_ab};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double t = wave_sum(v[q]);
        if (lane == 0) red[q][wid] = t;
    }
    __syncthreads();
    if (tid == 0) {
        double tot[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double acc = 0.0;
            for (int j = 0; j < kW; ++j) acc += red[q][j];
            tot[q] = acc;
        }
        const double W = tsum[0];
        const double va = tot[1] - tot[0] * tot[0] / W;
        const double vb = tsum[2] - tsum[1] * tsum[1] / W;
        const double cab = tot[2] - tot[0] * tsum[1] / W;
        const bool constant = k[0] == k[n - 1];    // one run of equal values
        float f;
        if (nan_flag[seg] || *target_nan) f = __builtin_nanf("");
        else if (constant || !(va > 0.0) || !(vb > 0.0) || !isfinite(va) || !isfinite(vb)) f = 0.0f;
        else f = static_cast<float>(fabs(cab / sqrt(va * vb)));
        fitness[prog0 + seg] = f;
    }
}

// k_stamp: one lane records the device's constant-rate clock (kernel timing
// inside a captured graph, where event records are not available).
__global__ __launch_bounds__(kWave) void k_stamp(uint64_t* __restrict__ out) {
    if (threadIdx.x == 0) out[0] = wall_clock64();
}

// ---------------------------------------------------------------------------
// Host side: scratch, launch configuration, entry points.
// ---------------------------------------------------------------------------

struct DeviceScratch {
    void* counter = nullptr;     // 256 bytes: the work counter
    int32_t* order = nullptr;
    size_t order_cap = 0;
    double* part = nullptr;
    size_t part_cap = 0;         // doubles
    double* ystat = nullptr;
    size_t ystat_cap = 0;        // doubles
    uint4* code = nullptr;       // the adjoint's instruction stream
    size_t code_cap = 0;         // instructions
    int32_t* clen = nullptr;
    size_t clen_cap = 0;
    uint4* ecode = nullptr;      // the evaluation kernel's instruction stream
    size_t ecode_cap = 0;
    int32_t* eclen = nullptr;
    size_t eclen_cap = 0;
    double* stats = nullptr;     // per-program statistics (kStats doubles each)
    size_t stats_cap = 0;
    double* gpart = nullptr;     // gradient partials
    size_t gpart_cap = 0;
    double* gextra = nullptr;    // gradient sums of constants beyond kGradLds
    size_t gextra_cap = 0;
    float* tape = nullptr;       // adjoint tape overflow
    size_t tape_cap = 0;
    float* fit_tmp = nullptr;
    size_t fit_tmp_cap = 0;
    // Spearman: sort keys (the first also takes the program outputs) and
    // carried values, double-buffered; the target's run starts, digit counts,
    // the target's ranks, NaN flags
    uint32_t* sp_k0 = nullptr;
    size_t sp_k0_cap = 0;
    uint32_t* sp_k1 = nullptr;
    size_t sp_k1_cap = 0;
    uint32_t* sp_v0 = nullptr;
    size_t sp_v0_cap = 0;
    uint32_t* sp_v1 = nullptr;
    size_t sp_v1_cap = 0;
    uint32_t* sp_rs = nullptr;
    size_t sp_rs_cap = 0;
    uint32_t* sp_cnt = nullptr;
    size_t sp_cnt_cap = 0;
    uint32_t* sp_r2y = nullptr;
    size_t sp_r2y_cap = 0;
    int32_t* sp_nan = nullptr;
    size_t sp_nan_cap = 0;
    double* sp_ty = nullptr;     // the target ranks' weighted sums (w, w b, w b^2)
    size_t sp_ty_cap = 0;
    int n_cu = 0;
    int dev = -1;
    std::string arch;
    bool fixed = false;          // carved from preallocated memory: never grown
};

std::mutex g_mu;
std::vector<DeviceScratch> g_dev;   // per-device arena of the plain entry points

// kernel timing (gp_profile_enable / gp_profile_read)
struct ProfRec {
    hipEvent_t a, b;
    int64_t node_rows;
};
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
gp_profile g_prof_acc{0, 0.0, 0};

gp_status grow(void** ptr, size_t* cap, size_t need_elems, size_t elem) {
    if (*cap >= need_elems && *ptr) return GP_OK;
    size_t n = std::max<size_t>(need_elems, 1);
    n = std::max(n, *cap * 2);
    if (*ptr) {
        GP_HIP(hipDeviceSynchronize());
        GP_HIP(hipFree(*ptr));
        *ptr = nullptr;
        *cap = 0;
    }
    hipError_t e = hipMalloc(ptr, n * elem);
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(GP_ERR_OUT_OF_MEMORY, std::string("scratch allocation: ") + hipGetErrorString(e));
    }
    *cap = n;
    return GP_OK;
}

gp_status scratch_init(DeviceScratch& s, int dev) {
    if (s.counter) return GP_OK;
    GP_HIP(hipMalloc(&s.counter, kCounterBytes));
    GP_HIP(hipMemset(s.counter, 0, kCounterBytes));
    hipDeviceProp_t prop;
    GP_HIP(hipGetDeviceProperties(&prop, dev));
    s.n_cu = prop.multiProcessorCount;
    s.dev = dev;
    s.arch = prop.gcnArchName;
    const size_t colon = s.arch.find(':');
    if (colon != std::string::npos) s.arch.resize(colon);
    return GP_OK;
}

bool scratch_empty(const DeviceScratch& s) {
    return !s.counter && !s.order && !s.part && !s.ystat && !s.code && !s.clen && !s.ecode && !s.eclen &&
           !s.stats && !s.gpart &&
           !s.gextra && !s.tape && !s.fit_tmp && !s.sp_k0 && !s.sp_k1 && !s.sp_v0 && !s.sp_v1 &&
           !s.sp_rs && !s.sp_cnt && !s.sp_r2y && !s.sp_nan && !s.sp_ty;
}

// Frees every buffer of s (the caller has made its device current and idle).
void scratch_free(DeviceScratch& s) {
    for (void* q : {s.counter, static_cast<void*>(s.order), static_cast<void*>(s.part),
                    static_cast<void*>(s.ystat), static_cast<void*>(s.code), static_cast<void*>(s.clen),
                    static_cast<void*>(s.ecode), static_cast<void*>(s.eclen),
                    static_cast<void*>(s.stats), static_cast<void*>(s.gpart), static_cast<void*>(s.gextra),
                    static_cast<void*>(s.tape), static_cast<void*>(s.fit_tmp),
                    static_cast<void*>(s.sp_k0), static_cast<void*>(s.sp_k1), static_cast<void*>(s.sp_v0),
                    static_cast<void*>(s.sp_v1), static_cast<void*>(s.sp_rs), static_cast<void*>(s.sp_cnt),
                    static_cast<void*>(s.sp_r2y), static_cast<void*>(s.sp_nan), static_cast<void*>(s.sp_ty)})
        if (q) (void)hipFree(q);
    s = DeviceScratch{};
}

// The shared arena of the current device.
gp_status arena(DeviceScratch** out) {
    int dev = 0;
    GP_HIP(hipGetDevice(&dev));
    if (static_cast<int>(g_dev.size()) <= dev) g_dev.resize(dev + 1);
    gp_status rc = scratch_init(g_dev[dev], dev);
    if (rc != GP_OK) return rc;
    *out = &g_dev[dev];
    return GP_OK;
}

gp_status check_pop(const gp_population_dev* pop, const char* who) {
    if (!pop) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": population is NULL");
    if (pop->n_programs < 0) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": n_programs < 0");
    if (pop->n_programs > 0 && (!pop->nodes || !pop->prog_off || !pop->const_off || !pop->len))
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": population pointer is NULL");
    if (pop->n_programs > 0 && pop->total_nodes < pop->n_programs)
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": total_nodes below n_programs");
    return GP_OK;
}

gp_status check_data(const gp_dataset_dev* d, const char* who, bool need_y) {
    if (!d) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": dataset is NULL");
    if (!d->X || d->n_features < 1)
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": dataset needs X and n_features >= 1");
    if (d->n_rows < 1) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": n_rows must be >= 1");
    if (d->ld < d->n_rows) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": ld below n_rows");
    if (need_y && !d->y) return fail(GP_ERR_INVALID_ARG, std::string(who) + ": y is NULL");
    return GP_OK;
}

gp_status check_fitness_metric(int metric, const char* who, bool spearman_ok = false) {
    if (gp_metric_larger_is_better(static_cast<gp_metric>(metric)) < 0)
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": unknown metric");
    if (metric >= GP_METRIC_USER_0 && metric <= GP_METRIC_USER_3 &&
        !((user_defined_mask() >> (GP_OP_USER2 + metric - GP_METRIC_USER_0)) & 1u))
        return fail(GP_ERR_INVALID_ARG, std::string(who) + ": a user loss needs its two-argument user function "
                                                            "(GP_OP_USER2 + i) defined");
    if (metric == GP_METRIC_SPEARMAN && !spearman_ok)
        return fail(GP_ERR_UNSUPPORTED, std::string(who) + ": Spearman has no derivative or launch configuration "
                                                            "(gp_fitness, generations and evolution compute it)");
    return GP_OK;
}

// ---------------------------------------------------------------------------
// Launch configuration of the evaluation kernel: forced > tuned > heuristic.
// ---------------------------------------------------------------------------
struct LaunchCfg {
    int R;        // rows per lane: 1, 2 or 4
    int freg;     // features held in registers: 0, 2 or 8
    int tiles;    // tiles of 64*R rows per chunk
    int wpb;      // wavefronts per block: 1, 2 or 4
};

bool cfg_valid(const LaunchCfg& c) {
    return (c.R == 1 || c.R == 2 || c.R == 4) && (c.freg == 0 || c.freg == 2 || c.freg == 8) && c.tiles >= 1 &&
           c.tiles <= (1 << 20) && (c.wpb == 1 || c.wpb == 2 || c.wpb == 4);
}

bool g_forced = false;
int64_t g_spear_workset = 0;       // Spearman batch working-set limit in bytes (0: automatic)
LaunchCfg g_forced_cfg{4, 0, 1, 4};

// Evaluation kernels differ by metric; each class is tuned on its own.
int kernel_class(int mode, int metric) {
    if (mode == 0) return 0;
    switch (metric) {
    case GP_METRIC_MSE:
    case GP_METRIC_RMSE: return 1;
    case GP_METRIC_MAE: return 2;
    case GP_METRIC_LOGLOSS: return 3;
    case GP_METRIC_PEARSON: return 4;
    default: return 5;   // user losses
    }
}

struct TuneKey {
    std::string arch;
    int n_cu;
    int F;
    int64_t N;
    int32_t P;
    int kclass;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, n_cu, F, N, P, kclass) < std::tie(o.arch, o.n_cu, o.F, o.N, o.P, o.kclass);
    }
};
struct TuneVal {
    LaunchCfg cfg;
    double ms;
};
std::map<TuneKey, TuneVal> g_tuned;

LaunchCfg heuristic_cfg(int F, int64_t N, int32_t P, int n_cu) {
    LaunchCfg c;
    c.R = 4;
    c.wpb = 4;
    // features in registers only for F <= 2: eight of them cost a wavefront of
    // occupancy at 4 rows per lane, which measures slower than reading them
    c.freg = F <= 2 ? 2 : 0;
    // a small job (fewer single-tile items than 8 per SIMD at 4 rows per
    // lane) takes one row per lane: four times the items, each a quarter as
    // long, so that the chip fills
    const int64_t tiles4 = (N + kWave * 4 - 1) / (kWave * 4);
    if (tiles4 * static_cast<int64_t>(P) < static_cast<int64_t>(n_cu) * 4 * 8) c.R = 1;
    const int64_t tile_rows = static_cast<int64_t>(kWave) * c.R;
    const int64_t n_tiles = (N + tile_rows - 1) / tile_rows;
    // aim for >= 32 work items per resident wavefront, chunks of <= 64 tiles
    const int64_t target_items = static_cast<int64_t>(n_cu) * 16 * 32;
    int64_t want_chunks = std::max<int64_t>(1, (target_items + P - 1) / std::max<int32_t>(P, 1));
    want_chunks = std::min(want_chunks, n_tiles);
    int64_t tiles = (n_tiles + want_chunks - 1) / want_chunks;
    tiles = std::min<int64_t>(std::max<int64_t>(tiles, 1), 64);
    c.tiles = static_cast<int>(tiles);
    return c;
}

LaunchCfg pick_cfg(const DeviceScratch& sc, int F, int64_t N, int32_t P, int kclass) {
    if (g_forced) return g_forced_cfg;
    auto it = g_tuned.find(TuneKey{sc.arch, sc.n_cu, F, N, P, kclass});
    if (it != g_tuned.end()) return it->second.cfg;
    return heuristic_cfg(F, N, P, sc.n_cu);
}

// How a launch of the evaluation kernel is timed: by the process-wide profile
// (plain entry points), by a pair of events recorded as graph nodes (captured
// generations), or not at all (autotuning, capture without timing).
struct Timing {
    bool profile = false;
    uint64_t* stamp = nullptr;   // device [2]: clock before and after the kernel
    const void** launched = nullptr;   // receives the evaluation kernel launched
};

template <int MODE, int METRIC>
gp_status launch_eval_m(const LaunchCfg& cfg, int n_cu, const PopView& pv, const CodeView& cv,
                        const DataView& dv, const Sched& s, float* out, double* part, hipStream_t st,
                        int64_t node_rows, const Timing& tm) {
    const int block = cfg.wpb * kWave;
    const size_t lds = static_cast<size_t>(cfg.wpb) * s.lds_slots * cfg.R * kWave * sizeof(float);
    auto go = [&](auto kernel) -> gp_status {
        int per_cu = 0;
        GP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds));
        per_cu = std::max(per_cu, 1);
        const int64_t waves_needed = (s.n_items + s.batch - 1) / s.batch;
        int64_t blocks = static_cast<int64_t>(per_cu) * n_cu;
        blocks = std::min<int64_t>(blocks, (waves_needed + cfg.wpb - 1) / cfg.wpb);
        blocks = std::max<int64_t>(blocks, 1);
        const bool prof = tm.profile && g_prof_on;
        ProfRec rec{nullptr, nullptr, node_rows};
        if (prof) {
            GP_HIP(hipEventCreate(&rec.a));
            GP_HIP(hipEventCreate(&rec.b));
            GP_HIP(hipEventRecord(rec.a, st));
        }
        if (tm.launched) *tm.launched = reinterpret_cast<const void*>(kernel);
        if (tm.stamp) hipLaunchKernelGGL(k_stamp, dim3(1), dim3(kWave), 0, st, tm.stamp);
        hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(blocks)), dim3(block), lds, st, pv, cv, dv, s, out,
                           part);
        GP_HIP(hipGetLastError());
        if (tm.stamp) {
            hipLaunchKernelGGL(k_stamp, dim3(1), dim3(kWave), 0, st, tm.stamp + 1);
            GP_HIP(hipGetLastError());
        }
        if (prof) {
            GP_HIP(hipEventRecord(rec.b, st));
            g_prof_pending.push_back(rec);
        }
        return GP_OK;
    };
#define GP_CASE(RR, FF)                                                \
    if (cfg.R == RR && cfg.freg == FF) return go(k_eval<RR, FF, MODE, METRIC>);
    GP_CASE(1, 0) GP_CASE(1, 2) GP_CASE(1, 8)
    GP_CASE(2, 0) GP_CASE(2, 2) GP_CASE(2, 8)
    GP_CASE(4, 0) GP_CASE(4, 2) GP_CASE(4, 8)
#undef GP_CASE
    return fail(GP_ERR_INVALID_ARG, "no kernel for this launch configuration");
}

gp_status launch_eval(int mode, int metric, const LaunchCfg& cfg, int n_cu, const PopView& pv,
                      const CodeView& cv, const DataView& dv, const Sched& s, float* out, double* part,
                      hipStream_t st, int64_t node_rows, const Timing& tm) {
    if (mode == 0)
        return launch_eval_m<0, GP_METRIC_MSE>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows, tm);
    switch (metric) {
    case GP_METRIC_MAE:
        return launch_eval_m<1, GP_METRIC_MAE>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows, tm);
    case GP_METRIC_MSE:
    case GP_METRIC_RMSE:
        return launch_eval_m<1, GP_METRIC_MSE>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows, tm);
    case GP_METRIC_LOGLOSS:
        return launch_eval_m<1, GP_METRIC_LOGLOSS>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows, tm);
    case GP_METRIC_PEARSON:
        return launch_eval_m<1, GP_METRIC_PEARSON>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows, tm);
    case GP_METRIC_USER_0:
    case GP_METRIC_USER_1:
    case GP_METRIC_USER_2:
    case GP_METRIC_USER_3:
        return launch_eval_m<1, GP_METRIC_USER_0>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows, tm);
    default: return fail(GP_ERR_UNSUPPORTED, "metric not supported by the fused fitness kernel");
    }
}

// How the evaluation stream expands user functions (Sec. V): the
// definitions, the loss wrapped around every program (GP_METRIC_USER_i), and
// the room this takes: program p's stream starts at prog_off[p] * mul +
// p * add, and the kernel's LDS holds lds_slots stack slots per row.
struct ExpandPlan {
    UserDefs defs;
    int32_t loss_fn = -1;
    int32_t mul = 1, add = 0;
    int32_t lds_slots = kEvalLds;
};

bool is_user_metric(int metric) { return metric >= GP_METRIC_USER_0 && metric <= GP_METRIC_USER_3; }

ExpandPlan expand_plan(int mode, int metric) {
    ExpandPlan x;
    user_defs(&x.defs);
    const uint32_t mask = user_defined_mask();
    if (mask == 0u) return x;
    for (int u = 0; u < kUserFns; ++u)
        if ((mask >> (GP_OP_USER1 + u)) & 1u) x.mul = std::max(x.mul, x.defs.len[u]);
    if (mode == 1 && is_user_metric(metric)) {
        x.loss_fn = metric - GP_METRIC_USER_0;
        x.add = 1 + x.defs.len[kUserFns / 2 + x.loss_fn];
    }
    x.lds_slots = kEvalLdsUser;
    return x;
}

// Scratch sizes one evaluation needs; grows sc's buffers to them (a fixed
// scratch must already hold them).  Called outside any stream capture (it may
// allocate).  The adjoint's instruction stream is reserved unless
// `adjoint_stream` is false.
gp_status reserve(DeviceScratch* sc, int32_t P, int64_t total_nodes, int64_t n_chunks, int mode, int metric,
                  bool adjoint_stream = true, int32_t ex_mul = 1, int32_t ex_add = 0) {
    auto need = [sc](auto** ptr, size_t* cap, size_t n, size_t elem) -> gp_status {
        if (!sc->fixed) return grow(reinterpret_cast<void**>(ptr), cap, n, elem);
        if (*ptr && *cap >= n) return GP_OK;
        return fail(GP_ERR_BUFFER_TOO_SMALL, "fixed scratch smaller than the evaluation needs");
    };
    gp_status rc = need(&sc->order, &sc->order_cap, P, sizeof(int32_t));
    if (rc != GP_OK) return rc;
    if (adjoint_stream) {
        rc = need(&sc->code, &sc->code_cap, static_cast<size_t>(total_nodes), sizeof(uint4));
        if (rc != GP_OK) return rc;
        rc = need(&sc->clen, &sc->clen_cap, P, sizeof(int32_t));
        if (rc != GP_OK) return rc;
    }
    // (+1: the evaluation kernel fetches one instruction past a program's end)
    rc = need(&sc->ecode, &sc->ecode_cap,
              static_cast<size_t>(total_nodes) * ex_mul + static_cast<size_t>(P) * ex_add + 1, sizeof(uint4));
    if (rc != GP_OK) return rc;
    rc = need(&sc->eclen, &sc->eclen_cap, P, sizeof(int32_t));
    if (rc != GP_OK) return rc;
    if (mode == 1) {
        const size_t kk = metric == GP_METRIC_PEARSON ? 4 : 1;
        rc = need(&sc->part, &sc->part_cap, static_cast<size_t>(P) * n_chunks * kk, sizeof(double));
        if (rc != GP_OK) return rc;
        rc = need(&sc->ystat, &sc->ystat_cap, static_cast<size_t>(n_chunks) * 4, sizeof(double));
        if (rc != GP_OK) return rc;
    }
    return GP_OK;
}

gp_status chunking(const gp_population_dev* pop, const gp_dataset_dev* data, const LaunchCfg& cfg,
                   int64_t* chunk, int64_t* n_chunks) {
    if (!cfg_valid(cfg)) return fail(GP_ERR_INVALID_ARG, "invalid launch configuration");
    if (cfg.freg > 0 && data->n_features > cfg.freg)
        return fail(GP_ERR_INVALID_ARG, "launch configuration holds fewer feature registers than n_features");
    *chunk = static_cast<int64_t>(cfg.tiles) * kWave * cfg.R;
    *n_chunks = (data->n_rows + *chunk - 1) / *chunk;
    // the 32-bit work counter overshoots n_items by at most one per wavefront
    if (*n_chunks * pop->n_programs > (int64_t{1} << 30))
        return fail(GP_ERR_INVALID_ARG, "too many work items (n_programs * row chunks above 2^30)");
    return GP_OK;
}

// Shared front half of the evaluation paths: configuration, scratch, the
// length ordering and the instruction streams.  `force` (nullable) overrides
// the configuration choice.  The evaluation kernel's stream (constant
// subtrees folded) is compiled unless `adjoint` asks for the adjoint's
// stream instead; `both` compiles the two (a backward pass that runs a
// forward pass first).
gp_status prepare(DeviceScratch* sc, const gp_population_dev* pop, const gp_dataset_dev* data, int mode,
                  int metric, hipStream_t st, const LaunchCfg* force, PopView* pv, CodeView* cvw, DataView* dv,
                  Sched* sch, LaunchCfg* cfg, bool adjoint = false, bool both = false) {
    *pv = PopView{pop->nodes, pop->prog_off, pop->consts, pop->const_off, pop->len, pop->n_programs};
    *dv = DataView{data->X, data->ld, data->n_features, data->n_rows, data->y, data->w};
    *cfg = force ? *force
                 : pick_cfg(*sc, data->n_features, data->n_rows, pop->n_programs, kernel_class(mode, metric));
    int64_t chunk = 0, n_chunks = 0;
    gp_status rc = chunking(pop, data, *cfg, &chunk, &n_chunks);
    if (rc != GP_OK) return rc;
    const ExpandPlan xp = expand_plan(mode, metric);
    rc = reserve(sc, pop->n_programs, pop->total_nodes, n_chunks, mode, metric, adjoint, xp.mul, xp.add);
    if (rc != GP_OK) return rc;
    // items claimed per atomic: enough that a launch issues about 32 claims
    // per resident wavefront (16 per CU), at most 8
    const int64_t n_items = n_chunks * pop->n_programs;
    const int64_t claims = static_cast<int64_t>(sc->n_cu) * 16 * 32;
    const int32_t batch = static_cast<int32_t>(std::min<int64_t>(8, std::max<int64_t>(1, n_items / claims)));
    *sch = Sched{chunk, static_cast<int32_t>(n_chunks), n_items, sc->order, static_cast<uint32_t*>(sc->counter),
                 batch, xp.lds_slots};
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(1024), 0, st, pop->len, pop->n_programs, sc->order,
                       static_cast<uint32_t*>(sc->counter));
    GP_HIP(hipGetLastError());
    const dim3 cgrid((pop->n_programs + kBlock - 1) / kBlock);
    if (!adjoint || both) {
        hipLaunchKernelGGL(k_compile_eval, cgrid, dim3(kBlock), 0, st, *pv, sc->ecode, sc->eclen, xp.defs,
                           xp.loss_fn, xp.mul, xp.add);
        GP_HIP(hipGetLastError());
    }
    if (adjoint) {
        hipLaunchKernelGGL(k_compile, cgrid, dim3(kBlock), 0, st, *pv, sc->code, sc->clen, 0);
        GP_HIP(hipGetLastError());
    }
    *cvw = CodeView{adjoint ? sc->code : nullptr, adjoint ? sc->clen : nullptr,
                    (!adjoint || both) ? sc->ecode : nullptr, (!adjoint || both) ? sc->eclen : nullptr, xp.mul,
                    xp.add};
    return GP_OK;
}

// Fitness of every program into `fitness` (device), on scratch sc.
gp_status fitness_impl(DeviceScratch* sc, const gp_population_dev* pop, const gp_dataset_dev* data, int metric,
                       float* fitness, hipStream_t st, const LaunchCfg* force, const Timing& tm) {
    PopView pv;
    CodeView cvw;
    DataView dv;
    Sched sch;
    LaunchCfg cfg;
    gp_status rc = prepare(sc, pop, data, 1, metric, st, force, &pv, &cvw, &dv, &sch, &cfg);
    if (rc != GP_OK) return rc;
    const bool need_ystats = data->w != nullptr || metric == GP_METRIC_PEARSON;
    if (need_ystats) {
        const int blocks = (sch.n_chunks + (kBlock / kWave) - 1) / (kBlock / kWave);
        hipLaunchKernelGGL(k_ystats, dim3(blocks), dim3(kBlock), 0, st, dv, sch.chunk, sch.n_chunks, sc->ystat);
        GP_HIP(hipGetLastError());
    }
    rc = launch_eval(1, metric, cfg, sc->n_cu, pv, cvw, dv, sch, nullptr, sc->part, st,
                     pop->total_nodes * data->n_rows, tm);
    if (rc != GP_OK) return rc;
    const int fblocks = (pop->n_programs + (kBlock / kWave) - 1) / (kBlock / kWave);
    const int has_w = data->w != nullptr;
#define GP_FIN(M)                                                                                  \
    hipLaunchKernelGGL(k_finalize<M>, dim3(fblocks), dim3(kBlock), 0, st, sc->part, sc->ystat,   \
                       sch.n_chunks, pop->n_programs, data->n_rows, has_w, fitness, nullptr)
    switch (metric) {
    case GP_METRIC_MAE: GP_FIN(GP_METRIC_MAE); break;
    case GP_METRIC_USER_0: case GP_METRIC_USER_1: case GP_METRIC_USER_2: case GP_METRIC_USER_3:
        GP_FIN(GP_METRIC_MAE);   // the weighted mean of the row losses
        break;
    case GP_METRIC_MSE: GP_FIN(GP_METRIC_MSE); break;
    case GP_METRIC_RMSE: GP_FIN(GP_METRIC_RMSE); break;
    case GP_METRIC_LOGLOSS: GP_FIN(GP_METRIC_LOGLOSS); break;
    default: GP_FIN(GP_METRIC_PEARSON); break;
    }
#undef GP_FIN
    GP_HIP(hipGetLastError());
    return GP_OK;
}

// ---- fitness without allocation ----
// One static array per device serves every gp_fitness_noalloc call on it.
// In host code `scratch` names a host-side stand-in: the device address comes
// from hipGetSymbolAddress, once per device, and only that address reaches
// kernels.
constexpr size_t kNoAllocBytes = size_t{64} << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kNoAllocMaxDevices = 64;
struct NoAllocDevice {
    unsigned char* ptr = nullptr;   // this device's copy of `scratch`
    int n_cu = 0;
    char arch[64] = {};
};
NoAllocDevice g_noalloc[kNoAllocMaxDevices];

size_t align256(size_t n) { return (n + 255) & ~size_t{255}; }

// Carves the scratch of one fitness evaluation out of the device's array into
// sc (caps exact, fixed: reserve() checks instead of growing).  Fails if the
// evaluation needs more than kNoAllocBytes.
gp_status noalloc_carve(unsigned char* base, DeviceScratch* sc, int32_t P, int64_t total_nodes, int64_t n_chunks,
                        int metric) {
    const size_t kk = metric == GP_METRIC_PEARSON ? 4 : 1;
    const ExpandPlan xp = expand_plan(1, metric);
    const size_t n_code = static_cast<size_t>(total_nodes) * xp.mul + static_cast<size_t>(P) * xp.add + 1;
    const size_t n_part = static_cast<size_t>(P) * static_cast<size_t>(n_chunks) * kk;
    const size_t n_ystat = static_cast<size_t>(n_chunks) * 4;
    const size_t bytes = kCounterBytes + align256(static_cast<size_t>(P) * sizeof(int32_t)) * 2 +
                         align256(n_code * sizeof(uint4)) + align256(n_part * sizeof(double)) +
                         align256(n_ystat * sizeof(double));
    if (bytes > kNoAllocBytes)
        return fail(GP_ERR_INVALID_ARG, "gp_fitness_noalloc: this evaluation needs " + std::to_string(bytes) +
                                            " bytes of scratch, above the limit of " +
                                            std::to_string(kNoAllocBytes) + " (use gp_fitness)");
    size_t off = 0;
    auto take = [&](size_t n) {
        unsigned char* q = base + off;
        off += align256(n);
        return q;
    };
    sc->counter = take(kCounterBytes);
    sc->order = reinterpret_cast<int32_t*>(take(static_cast<size_t>(P) * sizeof(int32_t)));
    sc->order_cap = static_cast<size_t>(P);
    sc->eclen = reinterpret_cast<int32_t*>(take(static_cast<size_t>(P) * sizeof(int32_t)));
    sc->eclen_cap = static_cast<size_t>(P);
    sc->ecode = reinterpret_cast<uint4*>(take(n_code * sizeof(uint4)));
    sc->ecode_cap = n_code;
    sc->part = reinterpret_cast<double*>(take(n_part * sizeof(double)));
    sc->part_cap = n_part;
    sc->ystat = reinterpret_cast<double*>(take(n_ystat * sizeof(double)));
    sc->ystat_cap = n_ystat;
    sc->fixed = true;
    return GP_OK;
}

gp_status tournament_impl(const float* fitness, const int32_t* len, int32_t P, int larger, float parsimony,
                          int32_t k, int32_t T, uint64_t seed, uint32_t gen, const uint32_t* gen_dev,
                          int32_t* winners, hipStream_t st) {
    if (T == 0) return GP_OK;
    const int blocks = (T + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_tournament, dim3(blocks), dim3(kBlock), 0, st, fitness, len, P, larger, parsimony, k, T,
                       seed, gen, gen_dev, winners);
    GP_HIP(hipGetLastError());
    return GP_OK;
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// Sorts the B segments of N float values at src (keys formed in the first
// pass, each carrying its row's target rank, or its row when rank2_y is
// NULL): the sorted keys and values end in k0 / v0, and nan_flag[s] is
// raised for a segment holding a NaN.  src may be k0 itself (the first pass
// writes k1 / v1 only).
gp_status radix_sort_segments(DeviceScratch* sc, const float* src, const uint32_t* rank2_y, int64_t N, int32_t B,
                              int32_t* nan_flag, hipStream_t st) {
    const int32_t T = static_cast<int32_t>((N + kRsTile - 1) / kRsTile);
    const uint32_t* in0 = reinterpret_cast<const uint32_t*>(src);
    hipLaunchKernelGGL(k_rs_count<true>, dim3(T, B), dim3(kRsBlock), 0, st, in0, N, T, 0, sc->sp_cnt, nan_flag);
    GP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rs_scan, dim3(B), dim3(1024), 0, st, sc->sp_cnt, T);
    GP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rs_scatter<true>, dim3(T, B), dim3(kRsScatterBlock), 0, st, in0, nullptr, sc->sp_k1,
                       sc->sp_v1, N, T, 0, sc->sp_cnt, rank2_y);
    GP_HIP(hipGetLastError());
    uint32_t *kin = sc->sp_k1, *vin = sc->sp_v1, *kout = sc->sp_k0, *vout = sc->sp_v0;
    for (int pass = 1; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_rs_count<false>, dim3(T, B), dim3(kRsBlock), 0, st, kin, N, T, shift, sc->sp_cnt,
                           nullptr);
        GP_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_rs_scan, dim3(B), dim3(1024), 0, st, sc->sp_cnt, T);
        GP_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_rs_scatter<false>, dim3(T, B), dim3(kRsScatterBlock), 0, st, kin, vin, kout, vout, N,
                           T, shift, sc->sp_cnt, nullptr);
        GP_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    return GP_OK;
}

// Spearman fitness (Sec. III-C3): programs in batches of B are evaluated,
// ranked by a sort, and correlated with the target's ranks.
gp_status spearman_impl(DeviceScratch* sc, const gp_population_dev* pop, const gp_dataset_dev* data,
                        float* fitness, hipStream_t st) {
    const int64_t N = data->n_rows;
    const int32_t P = pop->n_programs;
    if (N >= (int64_t{1} << 31)) return fail(GP_ERR_INVALID_ARG, "gp_fitness: Spearman needs n_rows below 2^31");
    const int32_t T = static_cast<int32_t>((N + kRsTile - 1) / kRsTile);
    // working set per program: keys and carried values twice, the outputs
    // sharing the first key buffer (16 bytes per row).  Up to the set limit,
    // else 16 GiB of it and at most half the
    // free memory; a program's fitness does not depend on its batch.  When
    // the programs need several batches, a batch is a whole number of rounds
    // of resident correlation workgroups (one per program).
    int64_t budget = g_spear_workset;
    if (budget <= 0) {
        size_t free_b = 0, total_b = 0;
        GP_HIP(hipMemGetInfo(&free_b, &total_b));
        budget = std::max<int64_t>(std::min<int64_t>(int64_t{16} << 30, static_cast<int64_t>(free_b / 2)),
                                   int64_t{256} << 20);
    }
    int64_t Bmax = std::max<int64_t>(1, budget / (16 * N));
    if (Bmax < P) {
        int per_cu = 0;
        GP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spear_corr<false>, 1024, 0));
        const int64_t round = static_cast<int64_t>(std::max(per_cu, 1)) * sc->n_cu;
        if (Bmax > round) Bmax = (Bmax / round) * round;
    }
    const int32_t B = static_cast<int32_t>(std::min<int64_t>(P, Bmax));
    const size_t BN = static_cast<size_t>(B) * static_cast<size_t>(N);
    gp_status rc = GP_OK;
    auto need = [&](void** ptr, size_t* cap, size_t n, size_t elem) {
        if (rc == GP_OK) rc = grow(ptr, cap, n, elem);
    };
    need(reinterpret_cast<void**>(&sc->sp_k0), &sc->sp_k0_cap, BN, sizeof(uint32_t));
    need(reinterpret_cast<void**>(&sc->sp_k1), &sc->sp_k1_cap, BN, sizeof(uint32_t));
    need(reinterpret_cast<void**>(&sc->sp_v0), &sc->sp_v0_cap, BN, sizeof(uint32_t));
    need(reinterpret_cast<void**>(&sc->sp_v1), &sc->sp_v1_cap, BN, sizeof(uint32_t));
    need(reinterpret_cast<void**>(&sc->sp_rs), &sc->sp_rs_cap, static_cast<size_t>(N), sizeof(uint32_t));
    need(reinterpret_cast<void**>(&sc->sp_cnt), &sc->sp_cnt_cap, static_cast<size_t>(B) * kRsRadix * T,
         sizeof(uint32_t));
    need(reinterpret_cast<void**>(&sc->sp_r2y), &sc->sp_r2y_cap, static_cast<size_t>(N), sizeof(uint32_t));
    need(reinterpret_cast<void**>(&sc->sp_nan), &sc->sp_nan_cap, static_cast<size_t>(B) + 1, sizeof(int32_t));
    need(reinterpret_cast<void**>(&sc->sp_ty), &sc->sp_ty_cap, 3, sizeof(double));
    if (rc != GP_OK) return rc;
    auto fill_nan_flags = [&](int32_t* flags, int32_t n) -> gp_status {
        hipLaunchKernelGGL(k_fill_i32, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, flags,
                           static_cast<int64_t>(n), 0);
        GP_HIP(hipGetLastError());
        return GP_OK;
    };
    // the target's ranks (twice the mean rank of each row); a NaN in the
    // target (flag B) makes every program's fitness NaN
    int32_t* target_nan = sc->sp_nan + B;
    if ((rc = fill_nan_flags(target_nan, 1)) != GP_OK) return rc;
    if ((rc = radix_sort_segments(sc, data->y, nullptr, N, 1, target_nan, st)) != GP_OK) return rc;
    hipLaunchKernelGGL(k_spear_rank_target, dim3(1), dim3(1024), 0, st, sc->sp_k0, sc->sp_v0, N, data->w,
                       sc->sp_rs, sc->sp_r2y, sc->sp_ty);
    GP_HIP(hipGetLastError());
    for (int32_t p0 = 0; p0 < P; p0 += B) {
        const int32_t b = std::min(B, P - p0);
        gp_population_dev view = *pop;
        view.prog_off = pop->prog_off + p0;
        view.const_off = pop->const_off + p0;
        view.len = pop->len + p0;
        view.n_programs = b;
        PopView pv;
        CodeView cvw;
        DataView dv;
        Sched sch;
        LaunchCfg cfg;
        rc = prepare(sc, &view, data, 0, GP_METRIC_MSE, st, nullptr, &pv, &cvw, &dv, &sch, &cfg);
        if (rc != GP_OK) return rc;
        // the outputs go to the first key buffer, which the sort's first pass
        // reads before anything writes it again
        float* out = reinterpret_cast<float*>(sc->sp_k0);
        rc = launch_eval(0, GP_METRIC_MSE, cfg, sc->n_cu, pv, cvw, dv, sch, out, nullptr, st, 0, Timing{});
        if (rc != GP_OK) return rc;
        if ((rc = fill_nan_flags(sc->sp_nan, b)) != GP_OK) return rc;
        if ((rc = radix_sort_segments(sc, out, data->w ? nullptr : sc->sp_r2y, N, b, sc->sp_nan, st)) != GP_OK)
            return rc;
        if (data->w)
            hipLaunchKernelGGL(k_spear_corr<true>, dim3(b), dim3(1024), 0, st, sc->sp_k0, sc->sp_v0, N, sc->sp_r2y,
                               data->w, sc->sp_ty, sc->sp_nan, target_nan, fitness, p0);
        else
            hipLaunchKernelGGL(k_spear_corr<false>, dim3(b), dim3(1024), 0, st, sc->sp_k0, sc->sp_v0, N, sc->sp_r2y,
                               nullptr, sc->sp_ty, sc->sp_nan, target_nan, fitness, p0);
        GP_HIP(hipGetLastError());
    }
    return GP_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate configurations of the fitness kernel on a prefix
// of at most kTuneRows rows and keeps the fastest for the full shape.
// ---------------------------------------------------------------------------
constexpr int64_t kTuneRows = int64_t{1} << 20;

gp_status autotune_impl(DeviceScratch* sc, const gp_population_dev* pop, const gp_dataset_dev* data, int metric,
                        int repeats, hipStream_t st, LaunchCfg* best_out, double* best_ms_out) {
    gp_dataset_dev sub = *data;
    sub.n_rows = std::min(data->n_rows, kTuneRows);
    gp_status rc = grow(reinterpret_cast<void**>(&sc->fit_tmp), &sc->fit_tmp_cap,
                        static_cast<size_t>(std::max(pop->n_programs, 1)), sizeof(float));
    if (rc != GP_OK) return rc;
    const LaunchCfg h = heuristic_cfg(data->n_features, data->n_rows, pop->n_programs, sc->n_cu);
    std::vector<int> fregs;
    if (data->n_features <= 2) fregs.push_back(2);
    if (data->n_features <= 8) fregs.push_back(8);
    fregs.push_back(0);
    std::vector<int> tiles;
    for (int t : {h.tiles / 4, h.tiles / 2, h.tiles, h.tiles * 2})
        if (t >= 1 && std::find(tiles.begin(), tiles.end(), t) == tiles.end()) tiles.push_back(t);
    hipEvent_t a = nullptr, b = nullptr;
    GP_HIP(hipEventCreate(&a));
    GP_HIP(hipEventCreate(&b));
    LaunchCfg best = h;
    double best_ms = -1.0;
    auto trial = [&](const LaunchCfg& c) {
        int64_t chunk = 0, n_chunks = 0;
        if (chunking(pop, data, c, &chunk, &n_chunks) != GP_OK) return;   // does not fit this shape
        double ms_min = -1.0;
        for (int rep = 0; rep <= repeats && rc == GP_OK; ++rep) {
            rc = hipEventRecord(a, st) == hipSuccess ? GP_OK : GP_ERR_DEVICE;
            if (rc == GP_OK) rc = fitness_impl(sc, pop, &sub, metric, sc->fit_tmp, st, &c, Timing{});
            if (rc == GP_OK) rc = hipEventRecord(b, st) == hipSuccess ? GP_OK : GP_ERR_DEVICE;
            if (rc == GP_OK) rc = hipEventSynchronize(b) == hipSuccess ? GP_OK : GP_ERR_DEVICE;
            float ms = 0.0f;
            if (rc == GP_OK) rc = hipEventElapsedTime(&ms, a, b) == hipSuccess ? GP_OK : GP_ERR_DEVICE;
            if (rc == GP_OK && rep > 0 && (ms_min < 0.0 || ms < ms_min)) ms_min = ms;  // rep 0 warms up
        }
        if (rc == GP_OK && ms_min >= 0.0 && (best_ms < 0.0 || ms_min < best_ms)) {
            best_ms = ms_min;
            best = c;
        }
    };
    // stage 1: rows per lane, feature registers, rows per work item (keeping
    // the heuristic's rows per item within a factor of 4), 4 waves per block
    for (int R : {1, 2, 4})
        for (int fr : fregs)
            for (int t : tiles)
                if (rc == GP_OK) trial(LaunchCfg{R, fr, std::max(1, t * 4 / R), 4});
    // stage 2: the block size for the best of stage 1
    const LaunchCfg s1 = best;
    for (int wpb : {1, 2})
        if (rc == GP_OK) trial(LaunchCfg{s1.R, s1.freg, s1.tiles, wpb});
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != GP_OK) return rc == GP_ERR_DEVICE ? fail(GP_ERR_DEVICE, "autotune: a timed launch failed") : rc;
    if (best_ms < 0.0) return fail(GP_ERR_INVALID_ARG, "autotune: no launch configuration fits this shape");
    g_tuned[TuneKey{sc->arch, sc->n_cu, data->n_features, data->n_rows, pop->n_programs, kernel_class(1, metric)}] =
        TuneVal{best, best_ms};
    *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return GP_OK;
}

// ---------------------------------------------------------------------------
// One generation as a HIP graph.
// ---------------------------------------------------------------------------
size_t align_up(size_t v) { return (v + 255) & ~size_t{255}; }

struct StageLayout {
    size_t gen, len, prog_off, const_off, nodes, consts, bytes;
};

StageLayout stage_layout(int32_t P, int64_t node_cap, int64_t const_cap) {
    StageLayout l;
    l.gen = 0;
    l.len = 256;
    l.prog_off = align_up(l.len + sizeof(int32_t) * static_cast<size_t>(P));
    l.const_off = align_up(l.prog_off + sizeof(int64_t) * (static_cast<size_t>(P) + 1));
    l.nodes = align_up(l.const_off + sizeof(int64_t) * (static_cast<size_t>(P) + 1));
    l.consts = align_up(l.nodes + sizeof(uint32_t) * static_cast<size_t>(node_cap));
    l.bytes = align_up(l.consts + sizeof(float) * static_cast<size_t>(std::max<int64_t>(const_cap, 1)));
    return l;
}

}  // namespace

struct gp_generation_s {
    gp_generation_params prm{};
    gp_dataset_dev data{};
    int dev = 0;
    hipStream_t stream = nullptr;
    DeviceScratch sc;
    StageLayout lay{};
    char* h_stage = nullptr;     // pinned: the population of the next generation
    char* d_stage = nullptr;
    float* d_fit = nullptr;
    int32_t* d_win = nullptr;
    float* h_fit = nullptr;      // pinned outputs
    int32_t* h_win = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t* d_stamp = nullptr;  // evaluation-kernel clock stamps (time_kernel)
    uint64_t* h_stamp = nullptr;
    int clock_khz = 0;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;   // event nodes around the evaluation kernel
    bool events = false;
    const void* eval_kernel = nullptr;
    LaunchCfg cfg{4, 0, 1};
    bool captured = false;
    double tuned_ms = -1.0;
    float kernel_ms = -1.0f;    // HIP events if inserted, else the clock stamps
    float clock_ms = -1.0f;     // clock stamps
};

namespace {

gp_population_dev stage_view(const gp_generation_s* g, int64_t total_nodes, int64_t total_consts) {
    gp_population_dev v{};
    v.nodes = reinterpret_cast<const uint32_t*>(g->d_stage + g->lay.nodes);
    v.prog_off = reinterpret_cast<const int64_t*>(g->d_stage + g->lay.prog_off);
    v.consts = reinterpret_cast<const float*>(g->d_stage + g->lay.consts);
    v.const_off = reinterpret_cast<const int64_t*>(g->d_stage + g->lay.const_off);
    v.len = reinterpret_cast<const int32_t*>(g->d_stage + g->lay.len);
    v.n_programs = g->prm.n_programs;
    v.total_nodes = total_nodes;
    v.max_len = 0;
    v.total_consts = total_consts;
    return v;
}

void generation_release(gp_generation_s* g) {
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ev_a) (void)hipEventDestroy(g->ev_a);
    if (g->ev_b) (void)hipEventDestroy(g->ev_b);
    if (g->d_stamp) (void)hipFree(g->d_stamp);
    if (g->h_stamp) (void)hipHostFree(g->h_stamp);
    if (g->h_stage) (void)hipHostFree(g->h_stage);
    if (g->h_fit) (void)hipHostFree(g->h_fit);
    if (g->h_win) (void)hipHostFree(g->h_win);
    if (g->d_stage) (void)hipFree(g->d_stage);
    if (g->d_fit) (void)hipFree(g->d_fit);
    if (g->d_win) (void)hipFree(g->d_win);
    scratch_free(g->sc);
    if (g->stream) (void)hipStreamDestroy(g->stream);
}

// Fitness step of the generation objects: the fused kernels, or for
// Spearman the batched evaluate / rank / correlate pipeline (whose buffers
// must exist before a capture: one eager call grows them).
gp_status graph_fitness(DeviceScratch* sc, const gp_population_dev* view, const gp_dataset_dev* data, int metric,
                        float* fit, hipStream_t st, const LaunchCfg* cfg, const Timing& tm) {
    if (metric == GP_METRIC_SPEARMAN) return spearman_impl(sc, view, data, fit, st);
    return fitness_impl(sc, view, data, metric, fit, st, cfg, tm);
}

// Records the generation into g->stream: population upload, fitness,
// tournament, result download.  Run under capture.
gp_status record_generation(gp_generation_s* g) {
    const gp_generation_params& p = g->prm;
    GP_HIP(hipMemcpyAsync(g->d_stage, g->h_stage, g->lay.bytes, hipMemcpyHostToDevice, g->stream));
    const gp_population_dev view = stage_view(g, p.node_capacity, p.const_capacity);
    Timing tm;
    tm.stamp = g->d_stamp;
    tm.launched = &g->eval_kernel;
    gp_status rc = graph_fitness(&g->sc, &view, &g->data, p.metric, g->d_fit, g->stream, &g->cfg, tm);
    if (rc != GP_OK) return rc;
    rc = tournament_impl(g->d_fit, view.len, p.n_programs, gp_metric_larger_is_better(static_cast<gp_metric>(p.metric)), p.parsimony,
                         p.tournament_size, p.n_tournaments, p.seed, 0,
                         reinterpret_cast<const uint32_t*>(g->d_stage + g->lay.gen), g->d_win, g->stream);
    if (rc != GP_OK) return rc;
    GP_HIP(hipMemcpyAsync(g->h_fit, g->d_fit, sizeof(float) * p.n_programs, hipMemcpyDeviceToHost, g->stream));
    if (p.n_tournaments > 0)
        GP_HIP(hipMemcpyAsync(g->h_win, g->d_win, sizeof(int32_t) * p.n_tournaments, hipMemcpyDeviceToHost,
                              g->stream));
    if (g->d_stamp)
        GP_HIP(hipMemcpyAsync(g->h_stamp, g->d_stamp, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, g->stream));
    return GP_OK;
}

// Puts event-record nodes right before and right after the evaluation-kernel
// node of a captured graph, so that the graph's launches record ev_a / ev_b
// around that kernel.  Returns false (graph unchanged or not) if HIP refuses;
// the caller then relies on the clock stamps.
bool insert_event_nodes(hipGraph_t graph, const void* func, hipEvent_t ev_a, hipEvent_t ev_b) {
    size_t n = 0;
    if (hipGraphGetNodes(graph, nullptr, &n) != hipSuccess || n == 0) return false;
    std::vector<hipGraphNode_t> nodes(n);
    if (hipGraphGetNodes(graph, nodes.data(), &n) != hipSuccess) return false;
    hipGraphNode_t K = nullptr;
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(nd, &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp{};
        if (hipGraphKernelNodeGetParams(nd, &kp) != hipSuccess) continue;
        if (kp.func == func) {
            if (K) return false;   // not unique
            K = nd;
        }
    }
    if (!K) return false;
    size_t nd_in = 0, nd_out = 0;
    if (hipGraphNodeGetDependencies(K, nullptr, &nd_in) != hipSuccess) return false;
    if (hipGraphNodeGetDependentNodes(K, nullptr, &nd_out) != hipSuccess) return false;
    std::vector<hipGraphNode_t> pred(nd_in), succ(nd_out);
    if (nd_in && hipGraphNodeGetDependencies(K, pred.data(), &nd_in) != hipSuccess) return false;
    if (nd_out && hipGraphNodeGetDependentNodes(K, succ.data(), &nd_out) != hipSuccess) return false;
    std::vector<hipGraphNode_t> Ks_in(nd_in, K), Ks_out(nd_out, K);
    hipGraphNode_t A = nullptr, B = nullptr;
    if (nd_in && hipGraphRemoveDependencies(graph, pred.data(), Ks_in.data(), nd_in) != hipSuccess) return false;
    if (hipGraphAddEventRecordNode(&A, graph, pred.data(), nd_in, ev_a) != hipSuccess) return false;
    if (hipGraphAddDependencies(graph, &A, &K, 1) != hipSuccess) return false;
    if (nd_out && hipGraphRemoveDependencies(graph, Ks_out.data(), succ.data(), nd_out) != hipSuccess) return false;
    if (hipGraphAddEventRecordNode(&B, graph, &K, 1, ev_b) != hipSuccess) return false;
    std::vector<hipGraphNode_t> Bs(nd_out, B);
    if (nd_out && hipGraphAddDependencies(graph, Bs.data(), succ.data(), nd_out) != hipSuccess) return false;
    return true;
}

// ---------------------------------------------------------------------------
// The device-resident loop: two alternating populations, a fitness history,
// the generation counter in device memory.
// ---------------------------------------------------------------------------
// History entry *gen - first: the fitness of every program and the
// population's node count (prog_off[P]).
__global__ void k_evo_record(const float* __restrict__ fit, int32_t P, const uint32_t* __restrict__ gen,
                             uint32_t first, int32_t cap, float* __restrict__ hist, int64_t* __restrict__ hist_nodes,
                             const int64_t* __restrict__ prog_off) {
    const uint32_t g = *gen - first;
    if (g >= static_cast<uint32_t>(cap)) return;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < P) hist[static_cast<int64_t>(g) * P + i] = fit[i];
    if (i == 0) hist_nodes[g] = prog_off[P];
}

// End of a generation: keep the mutation status bits, advance the counter.
__global__ void k_evo_step(uint32_t* __restrict__ gen, const int64_t* __restrict__ info,
                           unsigned long long* __restrict__ sticky) {
    if (threadIdx.x == 0) {
        *sticky |= static_cast<unsigned long long>(info[2]);
        *gen += 1u;
    }
}

// Sets the counter and the status word (a fill kernel: no memset node).
__global__ void k_evo_set(uint32_t* __restrict__ gen, uint32_t g, unsigned long long* __restrict__ sticky) {
    if (threadIdx.x == 0) {
        *gen = g;
        *sticky = 0ull;
    }
}

}  // namespace

struct EvoPop {
    uint32_t* nodes = nullptr;
    int64_t* prog_off = nullptr;
    float* consts = nullptr;
    int64_t* const_off = nullptr;
    int32_t* len = nullptr;
};

struct gp_evolution_s {
    gp_evolution_params prm{};
    gp_dataset_dev data{};
    int dev = 0;
    hipStream_t stream = nullptr;
    DeviceScratch sc;
    MutateWork mw;
    EvoPop pop[2];
    int64_t node_cap = 0, const_cap = 0;
    int cur = 0;                         // the current population
    float* d_fit = nullptr;
    int32_t* d_win = nullptr;            // [2P]
    int32_t* d_ops = nullptr;
    int32_t* d_first = nullptr;
    int32_t* d_nt = nullptr;
    int64_t* d_info = nullptr;           // [4]
    uint32_t* d_gen = nullptr;
    unsigned long long* d_sticky = nullptr;
    float* d_hist = nullptr;             // [(max_generations + 1) * P]
    int64_t* d_hist_nodes = nullptr;     // [max_generations + 1]
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    bool events = false;
    const void* eval_kernel = nullptr;
    LaunchCfg cfg{4, 0, 1};
    double tuned_ms = -1.0;
    float kernel_ms = -1.0f;
    int64_t generation = 0;              // generations run (host mirror of *d_gen)
    int64_t recorded = 0;                // history entries written
    bool captured = false;
};

namespace {

gp_population_dev evo_view(const gp_evolution_s* e, int which) {
    gp_population_dev v{};
    const EvoPop& q = e->pop[which];
    v.nodes = q.nodes;
    v.prog_off = q.prog_off;
    v.consts = q.consts;
    v.const_off = q.const_off;
    v.len = q.len;
    v.n_programs = e->prm.n_programs;
    v.total_nodes = e->node_cap;
    v.max_len = 0;
    v.total_consts = e->const_cap;
    return v;
}

void evolution_release(gp_evolution_s* e) {
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    for (int k = 0; k < 2; ++k) {
        if (e->exec[k]) (void)hipGraphExecDestroy(e->exec[k]);
        if (e->graph[k]) (void)hipGraphDestroy(e->graph[k]);
        EvoPop& q = e->pop[k];
        for (void* p : {static_cast<void*>(q.nodes), static_cast<void*>(q.prog_off), static_cast<void*>(q.consts),
                        static_cast<void*>(q.const_off), static_cast<void*>(q.len)})
            if (p) (void)hipFree(p);
        q = EvoPop{};
    }
    if (e->ev_a) (void)hipEventDestroy(e->ev_a);
    if (e->ev_b) (void)hipEventDestroy(e->ev_b);
    for (void* p : {static_cast<void*>(e->d_fit), static_cast<void*>(e->d_win), static_cast<void*>(e->d_ops),
                    static_cast<void*>(e->d_first), static_cast<void*>(e->d_nt), static_cast<void*>(e->d_info),
                    static_cast<void*>(e->d_gen), static_cast<void*>(e->d_sticky), static_cast<void*>(e->d_hist),
                    static_cast<void*>(e->d_hist_nodes)})
        if (p) (void)hipFree(p);
    mutate_work_free(&e->mw);
    scratch_free(e->sc);
    if (e->stream) (void)hipStreamDestroy(e->stream);
}

// Fitness of population `which` and its history entry (plain launches or
// under capture).
gp_status evo_evaluate(gp_evolution_s* e, int which, bool timed) {
    const gp_evolution_params& p = e->prm;
    const gp_population_dev v = evo_view(e, which);
    Timing tm;
    if (timed) tm.launched = &e->eval_kernel;
    gp_status rc = graph_fitness(&e->sc, &v, &e->data, p.metric, e->d_fit, e->stream, &e->cfg, tm);
    if (rc != GP_OK) return rc;
    const int32_t P = p.n_programs;
    hipLaunchKernelGGL(k_evo_record, dim3((P + 255) / 256), dim3(256), 0, e->stream, e->d_fit, P, e->d_gen,
                       static_cast<uint32_t>(p.first_generation), p.max_generations + 1, e->d_hist,
                       e->d_hist_nodes, v.prog_off);
    GP_HIP(hipGetLastError());
    return GP_OK;
}

// One generation from population a to population a ^ 1 (recorded under capture).
gp_status record_evolution(gp_evolution_s* e, int a) {
    const gp_evolution_params& p = e->prm;
    const int32_t P = p.n_programs;
    gp_status rc = evo_evaluate(e, a, true);
    if (rc != GP_OK) return rc;
    const gp_population_dev v = evo_view(e, a);
    rc = tournament_impl(e->d_fit, v.len, P, gp_metric_larger_is_better(static_cast<gp_metric>(p.metric)),
                         p.parsimony, p.tournament_size, 2 * P, p.tournament_seed, 0, e->d_gen, e->d_win, e->stream);
    if (rc != GP_OK) return rc;
    rc = plan_launch(p.evolve, P, 0, e->d_gen, e->d_ops, e->d_first, e->d_nt, e->stream);
    if (rc != GP_OK) return rc;
    const EvoPop& b = e->pop[a ^ 1];
    const gp_population_out_dev out{b.nodes, b.prog_off, b.consts, b.const_off, b.len, e->node_cap, e->const_cap};
    rc = mutate_launch(e->mw, p.evolve, p.init, v, e->d_ops, e->d_first, e->d_win, 2 * P, P, 0, e->d_gen, out,
                       e->d_info, e->stream);
    if (rc != GP_OK) return rc;
    hipLaunchKernelGGL(k_evo_step, dim3(1), dim3(64), 0, e->stream, e->d_gen, e->d_info, e->d_sticky);
    GP_HIP(hipGetLastError());
    return GP_OK;
}

gp_status evo_capture(gp_evolution_s* e, int a, bool with_events, bool* got_events) {
    *got_events = false;
    GP_HIP(hipStreamSynchronize(e->stream));
    GP_HIP(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
    gp_status rc = record_evolution(e, a);
    hipGraph_t graph = nullptr;
    const hipError_t err = hipStreamEndCapture(e->stream, &graph);
    if (rc != GP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (err != hipSuccess) return fail(GP_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(err));
    if (with_events) {
        if (!insert_event_nodes(graph, e->eval_kernel, e->ev_a, e->ev_b)) {
            // a half-edited graph is not used: capture again without events
            (void)hipGraphDestroy(graph);
            return evo_capture(e, a, false, got_events);
        }
        *got_events = true;
    }
    e->graph[a] = graph;
    return GP_OK;
}

}  // namespace

extern "C" {

void gp_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < g_dev.size(); ++d) {
        DeviceScratch& s = g_dev[d];
        if (scratch_empty(s)) continue;
        (void)hipSetDevice(static_cast<int>(d));
        (void)hipDeviceSynchronize();
        scratch_free(s);
    }
    (void)hipSetDevice(cur);
}

gp_status gp_get_launch_config(int32_t n_features, int64_t n_rows, int32_t n_programs, gp_metric metric,
                               gp_launch_config* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!out || n_features < 1 || n_rows < 1 || n_programs < 0)
        return fail(GP_ERR_INVALID_ARG, "gp_get_launch_config: bad arguments");
    gp_status rc = check_fitness_metric(metric, "gp_get_launch_config");
    if (rc != GP_OK) return rc;
    DeviceScratch* sc = nullptr;
    rc = arena(&sc);
    if (rc != GP_OK) return rc;
    const LaunchCfg c = pick_cfg(*sc, n_features, n_rows, n_programs, kernel_class(1, metric));
    *out = gp_launch_config{c.R, c.freg, c.tiles, c.wpb};
    return GP_OK;
}

gp_status gp_set_launch_config(const gp_launch_config* cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!cfg) {
        g_forced = false;
        return GP_OK;
    }
    const LaunchCfg c{cfg->rows_per_lane, cfg->feature_regs, cfg->tiles_per_chunk, cfg->waves_per_block};
    if (!cfg_valid(c))
        return fail(GP_ERR_INVALID_ARG, "gp_set_launch_config: rows_per_lane in {1,2,4}, feature_regs in {0,2,8}, "
                                        "tiles_per_chunk in [1, 2^20], waves_per_block in {1,2,4}");
    g_forced_cfg = c;
    g_forced = true;
    return GP_OK;
}

gp_status gp_set_spearman_workset(int64_t max_bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (max_bytes < 0) return fail(GP_ERR_INVALID_ARG, "gp_set_spearman_workset: max_bytes must be >= 0");
    g_spear_workset = max_bytes;
    return GP_OK;
}

gp_status gp_autotune(const gp_population_dev* pop, const gp_dataset_dev* data, gp_metric metric,
                      int32_t repeats, gp_launch_config* best, double* best_ms, void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    gp_status rc = check_pop(pop, "gp_autotune");
    if (rc != GP_OK) return rc;
    rc = check_data(data, "gp_autotune", true);
    if (rc != GP_OK) return rc;
    rc = check_fitness_metric(metric, "gp_autotune");
    if (rc != GP_OK) return rc;
    if (pop->n_programs < 1) return fail(GP_ERR_INVALID_ARG, "gp_autotune: empty population");
    if (repeats < 1 || repeats > 100) return fail(GP_ERR_INVALID_ARG, "gp_autotune: repeats in [1, 100]");
    DeviceScratch* sc = nullptr;
    rc = arena(&sc);
    if (rc != GP_OK) return rc;
    LaunchCfg c{};
    rc = autotune_impl(sc, pop, data, metric, repeats, static_cast<hipStream_t>(stream), &c, best_ms);
    if (rc != GP_OK) return rc;
    if (best) *best = gp_launch_config{c.R, c.freg, c.tiles, c.wpb};
    return GP_OK;
}

gp_status gp_autotune_save(const char* path) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!path) return fail(GP_ERR_INVALID_ARG, "gp_autotune_save: path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(GP_ERR_INVALID_ARG, std::string("gp_autotune_save: cannot open ") + path);
    for (const auto& kv : g_tuned) {
        const TuneKey& k = kv.first;
        const TuneVal& v = kv.second;
        std::fprintf(f,
                     "{\"arch\": \"%s\", \"n_cu\": %d, \"n_features\": %d, \"n_rows\": %lld, \"n_programs\": %d, "
                     "\"kernel\": %d, \"rows_per_lane\": %d, \"feature_regs\": %d, \"tiles_per_chunk\": %d, "
                     "\"waves_per_block\": %d, \"ms\": %.6f}\n",
                     k.arch.c_str(), k.n_cu, k.F, static_cast<long long>(k.N), k.P, k.kclass, v.cfg.R, v.cfg.freg,
                     v.cfg.tiles, v.cfg.wpb, v.ms);
    }
    const bool ok = std::fclose(f) == 0;
    return ok ? GP_OK : fail(GP_ERR_INVALID_ARG, "gp_autotune_save: write failed");
}

gp_status gp_autotune_load(const char* path) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!path) return fail(GP_ERR_INVALID_ARG, "gp_autotune_load: path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(GP_ERR_INVALID_ARG, std::string("gp_autotune_load: cannot open ") + path);
    std::vector<std::pair<TuneKey, TuneVal>> got;
    char line[1024];
    int lineno = 0;
    bool bad = false;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        if (line[0] == '\n' || line[0] == '\0') continue;
        char arch[64] = {0};
        int n_cu = 0, F = 0, P = 0, kc = 0, R = 0, fr = 0, t = 0, wpb = 0;
        long long N = 0;
        double ms = 0.0;
        const int n = std::sscanf(line,
                                  "{\"arch\": \"%63[^\"]\", \"n_cu\": %d, \"n_features\": %d, \"n_rows\": %lld, "
                                  "\"n_programs\": %d, \"kernel\": %d, \"rows_per_lane\": %d, \"feature_regs\": %d, "
                                  "\"tiles_per_chunk\": %d, \"waves_per_block\": %d, \"ms\": %lf}",
                                  arch, &n_cu, &F, &N, &P, &kc, &R, &fr, &t, &wpb, &ms);
        const LaunchCfg c{R, fr, t, wpb};
        if (n != 11 || !cfg_valid(c) || F < 1 || N < 1 || P < 0 || kc < 0 || kc > 4 ||
            (c.freg > 0 && F > c.freg)) {
            bad = true;
            break;
        }
        got.push_back({TuneKey{arch, n_cu, F, static_cast<int64_t>(N), P, kc}, TuneVal{c, ms}});
    }
    std::fclose(f);
    if (bad)
        return fail(GP_ERR_INVALID_ARG,
                    std::string("gp_autotune_load: malformed entry at line ") + std::to_string(lineno));
    for (auto& kv : got) g_tuned[kv.first] = kv.second;
    return GP_OK;
}

gp_status gp_autotune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned.clear();
    return GP_OK;
}

gp_status gp_profile_enable(int enable) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_prof_pending) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    g_prof_acc = gp_profile{0, 0.0, 0};
    g_prof_on = enable != 0;
    return GP_OK;
}

gp_status gp_profile_read(gp_profile* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!out) return fail(GP_ERR_INVALID_ARG, "gp_profile_read: out is NULL");
    for (auto& r : g_prof_pending) {
        GP_HIP(hipEventSynchronize(r.b));
        float ms = 0.0f;
        GP_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        g_prof_acc.launches += 1;
        g_prof_acc.total_ms += ms;
        g_prof_acc.node_rows += r.node_rows;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    *out = g_prof_acc;
    return GP_OK;
}

gp_status gp_evaluate(const gp_population_dev* pop, const gp_dataset_dev* data, float* out, void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    gp_status rc = check_pop(pop, "gp_evaluate");
    if (rc != GP_OK) return rc;
    rc = check_data(data, "gp_evaluate", false);
    if (rc != GP_OK) return rc;
    if (!out) return fail(GP_ERR_INVALID_ARG, "gp_evaluate: out is NULL");
    if (pop->n_programs == 0) return GP_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DeviceScratch* sc;
    rc = arena(&sc);
    if (rc != GP_OK) return rc;
    PopView pv;
    CodeView cvw;
    DataView dv;
    Sched sch;
    LaunchCfg cfg;
    rc = prepare(sc, pop, data, 0, GP_METRIC_MSE, st, nullptr, &pv, &cvw, &dv, &sch, &cfg);
    if (rc != GP_OK) return rc;
    Timing tm;
    tm.profile = true;
    return launch_eval(0, GP_METRIC_MSE, cfg, sc->n_cu, pv, cvw, dv, sch, out, nullptr, st,
                       pop->total_nodes * data->n_rows, tm);
}

gp_status gp_fitness(const gp_population_dev* pop, const gp_dataset_dev* data, gp_metric metric,
                     float* fitness, void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    gp_status rc = check_pop(pop, "gp_fitness");
    if (rc != GP_OK) return rc;
    rc = check_data(data, "gp_fitness", true);
    if (rc != GP_OK) return rc;
    if (!fitness) return fail(GP_ERR_INVALID_ARG, "gp_fitness: fitness is NULL");
    rc = check_fitness_metric(metric, "gp_fitness", true);
    if (rc != GP_OK) return rc;
    if (pop->n_programs == 0) return GP_OK;
    DeviceScratch* sc;
    rc = arena(&sc);
    if (rc != GP_OK) return rc;
    if (metric == GP_METRIC_SPEARMAN)
        return spearman_impl(sc, pop, data, fitness, static_cast<hipStream_t>(stream));
    Timing tm;
    tm.profile = true;
    return fitness_impl(sc, pop, data, metric, fitness, static_cast<hipStream_t>(stream), nullptr, tm);
}

gp_status gp_fitness_noalloc(const gp_population_dev* pop, const gp_dataset_dev* data, gp_metric metric,
                             float* fitness, void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    gp_status rc = check_pop(pop, "gp_fitness_noalloc");
    if (rc != GP_OK) return rc;
    rc = check_data(data, "gp_fitness_noalloc", true);
    if (rc != GP_OK) return rc;
    if (!fitness) return fail(GP_ERR_INVALID_ARG, "gp_fitness_noalloc: fitness is NULL");
    rc = check_fitness_metric(metric, "gp_fitness_noalloc");
    if (rc != GP_OK) return rc;
    if (pop->n_programs == 0) return GP_OK;
    int dev = 0;
    GP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(GP_ERR_UNSUPPORTED, "gp_fitness_noalloc: device index above the supported 64");
    NoAllocDevice& nd = g_noalloc[dev];
    if (!nd.ptr) {   // first call on this device (which is current)
        void* p = nullptr;
        GP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GP_ERR_DEVICE, "gp_fitness_noalloc: no device address for the scratch array");
        hipDeviceProp_t prop;
        GP_HIP(hipGetDeviceProperties(&prop, dev));
        nd.n_cu = prop.multiProcessorCount;
        size_t i = 0;
        for (; i + 1 < sizeof nd.arch && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
            nd.arch[i] = prop.gcnArchName[i];
        nd.arch[i] = 0;
        nd.ptr = static_cast<unsigned char*>(p);
    }
    DeviceScratch sc;
    sc.n_cu = nd.n_cu;
    sc.dev = dev;
    sc.arch = nd.arch;
    const LaunchCfg cfg = pick_cfg(sc, data->n_features, data->n_rows, pop->n_programs, kernel_class(1, metric));
    int64_t chunk = 0, n_chunks = 0;
    if ((rc = chunking(pop, data, cfg, &chunk, &n_chunks)) != GP_OK) return rc;
    if ((rc = noalloc_carve(nd.ptr, &sc, pop->n_programs, pop->total_nodes, n_chunks, metric)) != GP_OK)
        return rc;
    return fitness_impl(&sc, pop, data, metric, fitness, static_cast<hipStream_t>(stream), &cfg, Timing{});
}

gp_status gp_tournament(const float* fitness, const int32_t* len, int32_t n_programs, gp_metric metric,
                        float parsimony, int32_t tournament_size, int32_t n_tournaments, uint64_t seed,
                        uint64_t generation, int32_t* winners, void* stream) {
    if (n_programs < 1) return fail(GP_ERR_INVALID_ARG, "gp_tournament: n_programs must be >= 1");
    if (tournament_size < 1) return fail(GP_ERR_INVALID_ARG, "gp_tournament: tournament_size must be >= 1");
    if (n_tournaments < 0) return fail(GP_ERR_INVALID_ARG, "gp_tournament: n_tournaments < 0");
    if (generation > 0xffffffffull) return fail(GP_ERR_INVALID_ARG, "gp_tournament: generation above 2^32-1");
    const int larger = gp_metric_larger_is_better(metric);
    if (larger < 0) return fail(GP_ERR_INVALID_ARG, "gp_tournament: unknown metric");
    if (n_tournaments == 0) return GP_OK;
    if (!fitness || !len || !winners) return fail(GP_ERR_INVALID_ARG, "gp_tournament: NULL pointer");
    return tournament_impl(fitness, len, n_programs, larger, parsimony, tournament_size, n_tournaments, seed,
                           static_cast<uint32_t>(generation), nullptr, winners, static_cast<hipStream_t>(stream));
}

gp_status gp_generation_create(const gp_generation_params* prm, const gp_dataset_dev* data, gp_generation** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!prm || !out) return fail(GP_ERR_INVALID_ARG, "gp_generation_create: NULL argument");
    *out = nullptr;
    gp_status rc = check_data(data, "gp_generation_create", true);
    if (rc != GP_OK) return rc;
    rc = check_fitness_metric(prm->metric, "gp_generation_create", true);
    if (rc != GP_OK) return rc;
    if (prm->n_programs < 1 || prm->node_capacity < prm->n_programs || prm->const_capacity < 0 ||
        prm->tournament_size < 1 || prm->n_tournaments < 0 || prm->autotune < 0 || prm->time_kernel < 0)
        return fail(GP_ERR_INVALID_ARG, "gp_generation_create: bad sizes (n_programs >= 1, node_capacity >= "
                                        "n_programs, const_capacity >= 0, tournament_size >= 1, n_tournaments >= 0)");
    if (prm->node_capacity > (int64_t{1} << 32))
        return fail(GP_ERR_INVALID_ARG, "gp_generation_create: node_capacity above 2^32");
    auto* g = new (std::nothrow) gp_generation_s();
    if (!g) return fail(GP_ERR_OUT_OF_MEMORY, "gp_generation_create: out of host memory");
    g->prm = *prm;
    g->data = *data;
    g->lay = stage_layout(prm->n_programs, prm->node_capacity, prm->const_capacity);
    auto bail = [&](gp_status r) {
        generation_release(g);
        delete g;
        return r;
    };
    auto hip = [&](hipError_t e, const char* what) -> gp_status {
        return e == hipSuccess ? GP_OK : fail(GP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    if ((rc = hip(hipGetDevice(&g->dev), "hipGetDevice")) != GP_OK) return bail(rc);
    if ((rc = scratch_init(g->sc, g->dev)) != GP_OK) return bail(rc);
    if ((rc = hip(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking), "hipStreamCreate")) != GP_OK)
        return bail(rc);
    if ((rc = hip(hipHostMalloc(reinterpret_cast<void**>(&g->h_stage), g->lay.bytes, hipHostMallocDefault),
                  "hipHostMalloc")) != GP_OK)
        return bail(rc);
    std::memset(g->h_stage, 0, g->lay.bytes);
    if ((rc = hip(hipHostMalloc(reinterpret_cast<void**>(&g->h_fit), sizeof(float) * prm->n_programs,
                                hipHostMallocDefault), "hipHostMalloc")) != GP_OK)
        return bail(rc);
    if ((rc = hip(hipHostMalloc(reinterpret_cast<void**>(&g->h_win),
                                sizeof(int32_t) * std::max(prm->n_tournaments, 1), hipHostMallocDefault),
                  "hipHostMalloc")) != GP_OK)
        return bail(rc);
    if ((rc = hip(hipMalloc(reinterpret_cast<void**>(&g->d_stage), g->lay.bytes), "hipMalloc")) != GP_OK)
        return bail(rc == GP_ERR_DEVICE ? GP_ERR_OUT_OF_MEMORY : rc);
    if ((rc = hip(hipMalloc(reinterpret_cast<void**>(&g->d_fit), sizeof(float) * prm->n_programs), "hipMalloc")) !=
        GP_OK)
        return bail(rc);
    if ((rc = hip(hipMalloc(reinterpret_cast<void**>(&g->d_win), sizeof(int32_t) * std::max(prm->n_tournaments, 1)),
                  "hipMalloc")) != GP_OK)
        return bail(rc);
    if (prm->time_kernel) {
        if ((rc = hip(hipMalloc(reinterpret_cast<void**>(&g->d_stamp), 2 * sizeof(uint64_t)), "hipMalloc")) != GP_OK)
            return bail(rc);
        if ((rc = hip(hipHostMalloc(reinterpret_cast<void**>(&g->h_stamp), 2 * sizeof(uint64_t),
                                    hipHostMallocDefault), "hipHostMalloc")) != GP_OK)
            return bail(rc);
        if ((rc = hip(hipDeviceGetAttribute(&g->clock_khz, hipDeviceAttributeWallClockRate, g->dev),
                      "hipDeviceGetAttribute")) != GP_OK)
            return bail(rc);
        if (g->clock_khz <= 0) return bail(fail(GP_ERR_DEVICE, "gp_generation_create: no device wall clock rate"));
    }
    *out = g;
    return GP_OK;
}

gp_status gp_generation_run(gp_generation* g, const uint32_t* nodes, const int64_t* prog_off, const float* consts,
                            const int64_t* const_off, const int32_t* len, uint64_t generation, float* fitness_out,
                            int32_t* winners_out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g || !nodes || !prog_off || !const_off || !len)
        return fail(GP_ERR_INVALID_ARG, "gp_generation_run: NULL argument");
    const gp_generation_params& p = g->prm;
    const int32_t P = p.n_programs;
    if (generation > 0xffffffffull) return fail(GP_ERR_INVALID_ARG, "gp_generation_run: generation above 2^32-1");
    if (prog_off[0] != 0 || const_off[0] != 0)
        return fail(GP_ERR_INVALID_ARG, "gp_generation_run: offsets must start at 0");
    const int64_t total_nodes = prog_off[P];
    const int64_t total_consts = const_off[P];
    if (total_nodes > p.node_capacity || total_consts > p.const_capacity)
        return fail(GP_ERR_BUFFER_TOO_SMALL, "gp_generation_run: population exceeds the capacity given at creation");
    if (total_consts > 0 && !consts) return fail(GP_ERR_INVALID_ARG, "gp_generation_run: consts is NULL");
    for (int32_t q = 0; q < P; ++q)
        if (len[q] != prog_off[q + 1] - prog_off[q] || len[q] < 1 || const_off[q + 1] < const_off[q])
            return fail(GP_ERR_INVALID_ARG, "gp_generation_run: len / offsets are inconsistent at program " +
                                                std::to_string(q));
    // the device code assumes valid programs
    int32_t bad = -1;
    gp_status rc = gp_validate_population(nodes, prog_off, const_off, P, g->data.n_features, nullptr, &bad);
    if (rc != GP_OK) return rc;
    int cur = 0;
    GP_HIP(hipGetDevice(&cur));
    if (cur != g->dev) return fail(GP_ERR_INVALID_ARG, "gp_generation_run: another device is current");
    GP_HIP(hipStreamSynchronize(g->stream));
    // stage the population in pinned memory (one upload per generation)
    const uint32_t gen32 = static_cast<uint32_t>(generation);
    std::memcpy(g->h_stage + g->lay.gen, &gen32, sizeof gen32);
    std::memcpy(g->h_stage + g->lay.len, len, sizeof(int32_t) * P);
    std::memcpy(g->h_stage + g->lay.prog_off, prog_off, sizeof(int64_t) * (P + 1));
    std::memcpy(g->h_stage + g->lay.const_off, const_off, sizeof(int64_t) * (P + 1));
    std::memcpy(g->h_stage + g->lay.nodes, nodes, sizeof(uint32_t) * total_nodes);
    if (total_consts > 0) std::memcpy(g->h_stage + g->lay.consts, consts, sizeof(float) * total_consts);
    if (!g->captured) {
        // configuration: forced, tuned on this first population, or cached/heuristic
        const bool spear = p.metric == GP_METRIC_SPEARMAN;
        g->cfg = pick_cfg(g->sc, g->data.n_features, g->data.n_rows, P, kernel_class(spear ? 0 : 1, p.metric));
        if (p.autotune && !g_forced && !spear) {
            GP_HIP(hipMemcpyAsync(g->d_stage, g->h_stage, g->lay.bytes, hipMemcpyHostToDevice, g->stream));
            const gp_population_dev cur_view = stage_view(g, total_nodes, total_consts);
            rc = autotune_impl(&g->sc, &cur_view, &g->data, p.metric, 2, g->stream, &g->cfg, &g->tuned_ms);
            if (rc != GP_OK) return rc;
        }
        // every buffer the graph touches exists before capture
        int64_t chunk = 0, n_chunks = 0;
        const gp_population_dev cap_view = stage_view(g, p.node_capacity, p.const_capacity);
        rc = chunking(&cap_view, &g->data, g->cfg, &chunk, &n_chunks);
        if (rc != GP_OK) return rc;
        const ExpandPlan xp = expand_plan(1, p.metric);
        rc = reserve(&g->sc, P, p.node_capacity, n_chunks, 1, p.metric, true, xp.mul, xp.add);
        if (rc != GP_OK) return rc;
        if (spear) {
            // grow the Spearman buffers outside the capture (on this population)
            GP_HIP(hipMemcpyAsync(g->d_stage, g->h_stage, g->lay.bytes, hipMemcpyHostToDevice, g->stream));
            const gp_population_dev cap_full = stage_view(g, p.node_capacity, p.const_capacity);
            rc = spearman_impl(&g->sc, &cap_full, &g->data, g->d_fit, g->stream);
            if (rc != GP_OK) return rc;
        }
        GP_HIP(hipStreamSynchronize(g->stream));
        GP_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
        rc = record_generation(g);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(g->stream, &graph);
        if (rc != GP_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(GP_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        g->graph = graph;
        if (p.time_kernel) {
            GP_HIP(hipEventCreate(&g->ev_a));
            GP_HIP(hipEventCreate(&g->ev_b));
            g->events = insert_event_nodes(g->graph, g->eval_kernel, g->ev_a, g->ev_b);
            if (!g->events) {
                // a half-edited graph is not used: capture it again, stamps only
                (void)hipGraphDestroy(g->graph);
                g->graph = nullptr;
                GP_HIP(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
                rc = record_generation(g);
                const hipError_t e2 = hipStreamEndCapture(g->stream, &graph);
                if (rc != GP_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return rc;
                }
                if (e2 != hipSuccess)
                    return fail(GP_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
                g->graph = graph;
            }
        }
        GP_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        g->captured = true;
    }
    GP_HIP(hipGraphLaunch(g->exec, g->stream));
    GP_HIP(hipStreamSynchronize(g->stream));
    if (p.time_kernel && p.metric != GP_METRIC_SPEARMAN) {
        g->clock_ms = static_cast<float>(static_cast<double>(g->h_stamp[1] - g->h_stamp[0]) / g->clock_khz);
        g->kernel_ms = g->clock_ms;
        if (g->events) GP_HIP(hipEventElapsedTime(&g->kernel_ms, g->ev_a, g->ev_b));
    }
    if (fitness_out) std::memcpy(fitness_out, g->h_fit, sizeof(float) * P);
    if (winners_out && p.n_tournaments > 0) std::memcpy(winners_out, g->h_win, sizeof(int32_t) * p.n_tournaments);
    return GP_OK;
}

gp_status gp_generation_info(const gp_generation* g, gp_launch_config* cfg, float* kernel_ms, float* clock_ms,
                             int32_t* timed_by_events, double* tuned_ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g) return fail(GP_ERR_INVALID_ARG, "gp_generation_info: NULL generation");
    if (cfg) *cfg = gp_launch_config{g->cfg.R, g->cfg.freg, g->cfg.tiles, g->cfg.wpb};
    if (kernel_ms) *kernel_ms = g->kernel_ms;
    if (clock_ms) *clock_ms = g->clock_ms;
    if (timed_by_events) *timed_by_events = g->events ? 1 : 0;
    if (tuned_ms) *tuned_ms = g->tuned_ms;
    return GP_OK;
}

void gp_generation_destroy(gp_generation* g) {
    if (!g) return;
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->dev);
    generation_release(g);
    (void)hipSetDevice(cur);
    delete g;
}

gp_status gp_evolution_create(const gp_evolution_params* prm, const gp_dataset_dev* data, const uint32_t* nodes,
                              const int64_t* prog_off, const float* consts, const int64_t* const_off,
                              const int32_t* len, gp_evolution** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!prm || !out || !nodes || !prog_off || !const_off || !len)
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_create: NULL argument");
    *out = nullptr;
    gp_status rc = check_data(data, "gp_evolution_create", true);
    if (rc != GP_OK) return rc;
    rc = check_fitness_metric(prm->metric, "gp_evolution_create", true);
    if (rc != GP_OK) return rc;
    const int32_t P = prm->n_programs;
    if (P < 1 || P > (1 << 29) || prm->tournament_size < 1 || prm->max_generations < 1 ||
        prm->max_generations > (1 << 24) || prm->autotune < 0 || prm->time_kernel < 0)
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_create: need 1 <= n_programs <= 2^29, tournament_size >= 1, "
                                        "1 <= max_generations <= 2^24");
    rc = mutate_check(&prm->evolve, &prm->init, P, "gp_evolution_create");
    if (rc != GP_OK) return rc;
    if (prm->first_generation + static_cast<uint64_t>(prm->max_generations) > 0xffffffffull)
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_create: generation numbers above 2^32-1");
    if (prm->init.n_features != data->n_features)
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_create: init.n_features must equal the dataset's");
    if (prog_off[0] != 0 || const_off[0] != 0)
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_create: offsets must start at 0");
    int32_t longest = 1;
    for (int32_t q = 0; q < P; ++q) {
        if (len[q] != prog_off[q + 1] - prog_off[q] || len[q] < 1 || const_off[q + 1] < const_off[q])
            return fail(GP_ERR_INVALID_ARG, "gp_evolution_create: len / offsets are inconsistent at program " +
                                                std::to_string(q));
        longest = std::max(longest, len[q]);
    }
    if (const_off[P] > 0 && !consts) return fail(GP_ERR_INVALID_ARG, "gp_evolution_create: consts is NULL");
    rc = gp_validate_population(nodes, prog_off, const_off, P, data->n_features, nullptr, nullptr);
    if (rc != GP_OK) return rc;
    const int64_t lmax = std::max<int64_t>(prm->evolve.max_len, longest);
    const int64_t cap = static_cast<int64_t>(P) * lmax;
    if (cap > (int64_t{1} << 32))
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_create: n_programs * max length above 2^32 nodes");
    auto* e = new (std::nothrow) gp_evolution_s();
    if (!e) return fail(GP_ERR_OUT_OF_MEMORY, "gp_evolution_create: out of host memory");
    e->prm = *prm;
    e->data = *data;
    e->node_cap = cap;
    e->const_cap = cap;
    auto bail = [&](gp_status r) {
        evolution_release(e);
        delete e;
        return r;
    };
    auto hip = [&](hipError_t err, const char* what) -> gp_status {
        return err == hipSuccess ? GP_OK : fail(GP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(err));
    };
    auto dmalloc = [&](void** ptr, size_t bytes) -> gp_status {
        return hipMalloc(ptr, std::max<size_t>(bytes, 4)) == hipSuccess
                   ? GP_OK
                   : fail(GP_ERR_OUT_OF_MEMORY, "gp_evolution_create: hipMalloc failed");
    };
    if ((rc = hip(hipGetDevice(&e->dev), "hipGetDevice")) != GP_OK) return bail(rc);
    if ((rc = scratch_init(e->sc, e->dev)) != GP_OK) return bail(rc);
    if ((rc = hip(hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking), "hipStreamCreate")) != GP_OK)
        return bail(rc);
    for (int k = 0; k < 2; ++k) {
        EvoPop& q = e->pop[k];
        if ((rc = dmalloc(reinterpret_cast<void**>(&q.nodes), sizeof(uint32_t) * cap)) != GP_OK) return bail(rc);
        if ((rc = dmalloc(reinterpret_cast<void**>(&q.consts), sizeof(float) * cap)) != GP_OK) return bail(rc);
        if ((rc = dmalloc(reinterpret_cast<void**>(&q.prog_off), sizeof(int64_t) * (P + 1))) != GP_OK) return bail(rc);
        if ((rc = dmalloc(reinterpret_cast<void**>(&q.const_off), sizeof(int64_t) * (P + 1))) != GP_OK)
            return bail(rc);
        if ((rc = dmalloc(reinterpret_cast<void**>(&q.len), sizeof(int32_t) * P)) != GP_OK) return bail(rc);
    }
    const size_t hist_n = static_cast<size_t>(prm->max_generations + 1);
    if ((rc = dmalloc(reinterpret_cast<void**>(&e->d_fit), sizeof(float) * P)) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_win), sizeof(int32_t) * 2 * P)) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_ops), sizeof(int32_t) * P)) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_first), sizeof(int32_t) * P)) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_nt), sizeof(int32_t))) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_info), sizeof(int64_t) * 4)) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_gen), sizeof(uint32_t))) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_sticky), sizeof(unsigned long long))) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_hist), sizeof(float) * hist_n * P)) != GP_OK ||
        (rc = dmalloc(reinterpret_cast<void**>(&e->d_hist_nodes), sizeof(int64_t) * hist_n)) != GP_OK)
        return bail(rc);
    if ((rc = mutate_work_reserve(&e->mw, P, prm->init)) != GP_OK) return bail(rc);
    // the initial population
    const EvoPop& q0 = e->pop[0];
    if ((rc = hip(hipMemcpy(q0.nodes, nodes, sizeof(uint32_t) * prog_off[P], hipMemcpyHostToDevice), "hipMemcpy")) !=
            GP_OK ||
        (const_off[P] > 0 &&
         (rc = hip(hipMemcpy(q0.consts, consts, sizeof(float) * const_off[P], hipMemcpyHostToDevice), "hipMemcpy")) !=
             GP_OK) ||
        (rc = hip(hipMemcpy(q0.prog_off, prog_off, sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice), "hipMemcpy")) !=
            GP_OK ||
        (rc = hip(hipMemcpy(q0.const_off, const_off, sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice),
                  "hipMemcpy")) != GP_OK ||
        (rc = hip(hipMemcpy(q0.len, len, sizeof(int32_t) * P, hipMemcpyHostToDevice), "hipMemcpy")) != GP_OK)
        return bail(rc);
    hipLaunchKernelGGL(k_evo_set, dim3(1), dim3(64), 0, e->stream, e->d_gen,
                       static_cast<uint32_t>(prm->first_generation), e->d_sticky);
    if ((rc = hip(hipGetLastError(), "k_evo_set")) != GP_OK) return bail(rc);
    if ((rc = hip(hipStreamSynchronize(e->stream), "hipStreamSynchronize")) != GP_OK) return bail(rc);
    *out = e;
    return GP_OK;
}

namespace {
gp_status evo_prepare(gp_evolution_s* e) {
    if (e->captured) return GP_OK;
    const gp_evolution_params& p = e->prm;
    const int32_t P = p.n_programs;
    const bool spear = p.metric == GP_METRIC_SPEARMAN;
    e->cfg = pick_cfg(e->sc, e->data.n_features, e->data.n_rows, P, kernel_class(spear ? 0 : 1, p.metric));
    if (p.autotune && !g_forced && !spear) {
        const gp_population_dev v = evo_view(e, e->cur);
        gp_status rc = autotune_impl(&e->sc, &v, &e->data, p.metric, 2, e->stream, &e->cfg, &e->tuned_ms);
        if (rc != GP_OK) return rc;
    }
    int64_t chunk = 0, n_chunks = 0;
    const gp_population_dev v = evo_view(e, 0);
    gp_status rc = chunking(&v, &e->data, e->cfg, &chunk, &n_chunks);
    if (rc != GP_OK) return rc;
    const ExpandPlan xp = expand_plan(1, p.metric);
    rc = reserve(&e->sc, P, e->node_cap, n_chunks, 1, p.metric, true, xp.mul, xp.add);
    if (rc != GP_OK) return rc;
    if (spear) {
        // grow the Spearman buffers outside the capture (on the current population)
        const gp_population_dev vc = evo_view(e, e->cur);
        rc = spearman_impl(&e->sc, &vc, &e->data, e->d_fit, e->stream);
        if (rc != GP_OK) return rc;
        GP_HIP(hipStreamSynchronize(e->stream));
    }
    if (p.time_kernel) {
        GP_HIP(hipEventCreate(&e->ev_a));
        GP_HIP(hipEventCreate(&e->ev_b));
    }
    // events count only if both graphs carry them
    bool events = p.time_kernel != 0;
    for (int a = 0; a < 2; ++a) {
        bool got = false;
        rc = evo_capture(e, a, p.time_kernel != 0, &got);
        if (rc != GP_OK) return rc;
        events = events && got;
        GP_HIP(hipGraphInstantiate(&e->exec[a], e->graph[a], nullptr, nullptr, 0));
    }
    e->events = events;
    e->captured = true;
    return GP_OK;
}
}  // namespace

gp_status gp_evolution_run(gp_evolution* e, int32_t n) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!e || n < 0) return fail(GP_ERR_INVALID_ARG, "gp_evolution_run: bad arguments");
    if (e->generation + n > e->prm.max_generations)
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_run: beyond max_generations");
    int cur_dev = 0;
    GP_HIP(hipGetDevice(&cur_dev));
    if (cur_dev != e->dev) return fail(GP_ERR_INVALID_ARG, "gp_evolution_run: another device is current");
    gp_status rc = evo_prepare(e);
    if (rc != GP_OK) return rc;
    for (int32_t k = 0; k < n; ++k) {
        GP_HIP(hipGraphLaunch(e->exec[e->cur], e->stream));
        e->cur ^= 1;
    }
    GP_HIP(hipStreamSynchronize(e->stream));
    e->generation += n;
    e->recorded = std::max(e->recorded, e->generation);
    unsigned long long sticky = 0;
    GP_HIP(hipMemcpy(&sticky, e->d_sticky, sizeof sticky, hipMemcpyDeviceToHost));
    if (n > 0 && e->events) GP_HIP(hipEventElapsedTime(&e->kernel_ms, e->ev_a, e->ev_b));
    if (sticky)
        return fail(GP_ERR_DEVICE, "gp_evolution_run: mutation status bits " + std::to_string(sticky) +
                                       " (1 capacity, 2 index out of range, 4 donor bound)");
    return GP_OK;
}

gp_status gp_evolution_evaluate(gp_evolution* e) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!e) return fail(GP_ERR_INVALID_ARG, "gp_evolution_evaluate: NULL");
    if (e->generation > e->prm.max_generations)
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_evaluate: beyond max_generations");
    gp_status rc = evo_prepare(e);
    if (rc != GP_OK) return rc;
    rc = evo_evaluate(e, e->cur, false);
    if (rc != GP_OK) return rc;
    GP_HIP(hipStreamSynchronize(e->stream));
    e->recorded = std::max(e->recorded, e->generation + 1);
    return GP_OK;
}

gp_status gp_evolution_history(const gp_evolution* e, int32_t capacity, int32_t* n_recorded, float* fitness_history,
                               int64_t* nodes_history) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!e || capacity < 0) return fail(GP_ERR_INVALID_ARG, "gp_evolution_history: bad arguments");
    if (n_recorded) *n_recorded = static_cast<int32_t>(e->recorded);
    const int64_t n = std::min<int64_t>(capacity, e->recorded);
    const int64_t P = e->prm.n_programs;
    GP_HIP(hipStreamSynchronize(e->stream));
    if (fitness_history && n > 0)
        GP_HIP(hipMemcpy(fitness_history, e->d_hist, sizeof(float) * n * P, hipMemcpyDeviceToHost));
    if (nodes_history && n > 0)
        GP_HIP(hipMemcpy(nodes_history, e->d_hist_nodes, sizeof(int64_t) * n, hipMemcpyDeviceToHost));
    return GP_OK;
}

gp_status gp_evolution_population(const gp_evolution* e, uint32_t* nodes, int64_t nodes_cap, int64_t* prog_off,
                                  float* consts, int64_t consts_cap, int64_t* const_off, int32_t* len,
                                  int64_t* total_nodes, int64_t* total_consts) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!e || !prog_off || !const_off || !len || !total_nodes || !total_consts)
        return fail(GP_ERR_INVALID_ARG, "gp_evolution_population: NULL argument");
    const int32_t P = e->prm.n_programs;
    const EvoPop& q = e->pop[e->cur];
    GP_HIP(hipStreamSynchronize(e->stream));
    GP_HIP(hipMemcpy(prog_off, q.prog_off, sizeof(int64_t) * (P + 1), hipMemcpyDeviceToHost));
    GP_HIP(hipMemcpy(const_off, q.const_off, sizeof(int64_t) * (P + 1), hipMemcpyDeviceToHost));
    GP_HIP(hipMemcpy(len, q.len, sizeof(int32_t) * P, hipMemcpyDeviceToHost));
    *total_nodes = prog_off[P];
    *total_consts = const_off[P];
    if (*total_nodes > nodes_cap || *total_consts > consts_cap || !nodes || (*total_consts > 0 && !consts))
        return fail(GP_ERR_BUFFER_TOO_SMALL, "gp_evolution_population: a capacity is short");
    GP_HIP(hipMemcpy(nodes, q.nodes, sizeof(uint32_t) * *total_nodes, hipMemcpyDeviceToHost));
    if (*total_consts > 0) GP_HIP(hipMemcpy(consts, q.consts, sizeof(float) * *total_consts, hipMemcpyDeviceToHost));
    return GP_OK;
}

gp_status gp_evolution_info(const gp_evolution* e, gp_launch_config* cfg, float* kernel_ms, int64_t* generation,
                            double* tuned_ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!e) return fail(GP_ERR_INVALID_ARG, "gp_evolution_info: NULL");
    if (cfg) *cfg = gp_launch_config{e->cfg.R, e->cfg.freg, e->cfg.tiles, e->cfg.wpb};
    if (kernel_ms) *kernel_ms = e->events ? e->kernel_ms : -1.0f;
    if (generation) *generation = e->generation;
    if (tuned_ms) *tuned_ms = e->tuned_ms;
    return GP_OK;
}

void gp_evolution_destroy(gp_evolution* e) {
    if (!e) return;
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(e->dev);
    evolution_release(e);
    (void)hipSetDevice(cur);
    delete e;
}

gp_status gp_fitness_backward(const gp_population_dev* pop, const gp_dataset_dev* data, gp_metric metric,
                              const float* grad_fitness, float* fitness_out, float* grad_consts,
                              void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    gp_status rc = check_pop(pop, "gp_fitness_backward");
    if (rc != GP_OK) return rc;
    rc = check_data(data, "gp_fitness_backward", true);
    if (rc != GP_OK) return rc;
    rc = check_fitness_metric(metric, "gp_fitness_backward");
    if (rc != GP_OK) return rc;
    if (is_user_metric(metric))
        return fail(GP_ERR_UNSUPPORTED, "gp_fitness_backward: user losses have no derivative here");
    if (pop->n_programs == 0) return GP_OK;
    if (pop->total_consts < 0 || (pop->total_consts > 0 && (!grad_consts || !pop->consts)))
        return fail(GP_ERR_INVALID_ARG, "gp_fitness_backward: grad_consts and consts are needed");
    if (pop->max_len < 1)
        return fail(GP_ERR_INVALID_ARG, "gp_fitness_backward: max_len must bound the program lengths");
    if (pop->max_len > kMaxAdjointLen)
        return fail(GP_ERR_INVALID_ARG, "gp_fitness_backward: programs longer than 2^25 nodes are not supported");
    hipStream_t st = static_cast<hipStream_t>(stream);
    DeviceScratch* sc;
    rc = arena(&sc);
    if (rc != GP_OK) return rc;
    if (user_defined_mask() != 0u) {
        // user functions have no derivative here: look for them (this
        // waits for the stream)
        uint32_t* flag = static_cast<uint32_t*>(sc->counter) + kFlagWord;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, flag);
        GP_HIP(hipGetLastError());
        const int64_t nb = std::min<int64_t>((pop->total_nodes + kBlock - 1) / kBlock, 4096);
        hipLaunchKernelGGL(k_find_user, dim3(static_cast<unsigned>(std::max<int64_t>(nb, 1))), dim3(kBlock), 0, st,
                           pop->nodes, pop->total_nodes, flag);
        GP_HIP(hipGetLastError());
        uint32_t found = 0u;
        GP_HIP(hipMemcpyAsync(&found, flag, sizeof found, hipMemcpyDeviceToHost, st));
        GP_HIP(hipStreamSynchronize(st));
        if (found)
            return fail(GP_ERR_UNSUPPORTED, "gp_fitness_backward: the population uses user functions, which have "
                                            "no derivative here");
    }
    PopView pv;
    CodeView cvw;
    DataView dv;
    Sched sch;
    LaunchCfg cfg;
    // the adjoint's stream (no constant folding: every constant carries its
    // own derivative); RMSE and Pearson also run the evaluation kernel first
    const bool needs_forward = metric == GP_METRIC_RMSE || metric == GP_METRIC_PEARSON;
    rc = prepare(sc, pop, data, 1, metric, st, nullptr, &pv, &cvw, &dv, &sch, &cfg, true, needs_forward);
    if (rc != GP_OK) return rc;
    const int32_t P = pop->n_programs;
    const int64_t nc = std::max<int64_t>(pop->total_consts, 1);
    // rows per lane of the adjoint: a forced configuration's, else the one
    // (2 or 4) that keeps more rows in flight per CU (below)
    const int RA = g_forced ? g_forced_cfg.R : 0;
    const int64_t tape_max = 2 * static_cast<int64_t>(pop->max_len) + 2;   // tape entries per wavefront
    rc = grow(reinterpret_cast<void**>(&sc->stats), &sc->stats_cap, static_cast<size_t>(P) * kStats + 1,
              sizeof(double));
    if (rc != GP_OK) return rc;
    rc = grow(reinterpret_cast<void**>(&sc->gpart), &sc->gpart_cap, static_cast<size_t>(nc) * sch.n_chunks,
              sizeof(double));
    if (rc != GP_OK) return rc;
    rc = grow(reinterpret_cast<void**>(&sc->gextra), &sc->gextra_cap, static_cast<size_t>(nc), sizeof(double));
    if (rc != GP_OK) return rc;
    rc = grow(reinterpret_cast<void**>(&sc->fit_tmp), &sc->fit_tmp_cap, static_cast<size_t>(P), sizeof(float));
    if (rc != GP_OK) return rc;
    double* wsum = sc->stats + static_cast<size_t>(P) * kStats;
    const int has_w = data->w != nullptr;
    const int ys_blocks = (sch.n_chunks + (kBlock / kWave) - 1) / (kBlock / kWave);
    hipLaunchKernelGGL(k_ystats, dim3(ys_blocks), dim3(kBlock), 0, st, dv, sch.chunk, sch.n_chunks, sc->ystat);
    GP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_wsum, dim3(1), dim3(kWave), 0, st, sc->ystat, sch.n_chunks, has_w, data->n_rows, wsum);
    GP_HIP(hipGetLastError());
    const int fblocks = (P + (kBlock / kWave) - 1) / (kBlock / kWave);
    float* fit = fitness_out ? fitness_out : sc->fit_tmp;
    if (needs_forward) {
        rc = launch_eval(1, metric, cfg, sc->n_cu, pv, cvw, dv, sch, nullptr, sc->part, st,
                         pop->total_nodes * data->n_rows, Timing{});
        if (rc != GP_OK) return rc;
        if (metric == GP_METRIC_RMSE)
            hipLaunchKernelGGL(k_finalize<GP_METRIC_RMSE>, dim3(fblocks), dim3(kBlock), 0, st, sc->part, sc->ystat,
                               sch.n_chunks, P, data->n_rows, has_w, fit, sc->stats);
        else
            hipLaunchKernelGGL(k_finalize<GP_METRIC_PEARSON>, dim3(fblocks), dim3(kBlock), 0, st, sc->part,
                               sc->ystat, sch.n_chunks, P, data->n_rows, has_w, fit, sc->stats);
        GP_HIP(hipGetLastError());
        // the forward pass consumed the work counter: reset it (and reorder)
        hipLaunchKernelGGL(k_prepare, dim3(1), dim3(1024), 0, st, pop->len, P, sc->order,
                           static_cast<uint32_t*>(sc->counter));
        GP_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>((nc + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       sc->gextra, nc);
    GP_HIP(hipGetLastError());
    // features in registers when they fit -- unless a forced configuration
    // says otherwise, or holding them would cost a wavefront of occupancy
    // against reading them from memory (the choice below, per kernel)
    const int freg_fit = data->n_features <= 2 ? 2 : (data->n_features <= 8 ? 8 : 0);
    const int freg = (g_forced && g_forced_cfg.freg == 0) ? 0 : freg_fit;
    auto occ = [](const void* k) {
        int n = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kWave, 0);
        return n;
    };
    double* lossp = needs_forward ? nullptr : sc->part;
    auto go = [&](auto kernel, int64_t wave_floats) -> gp_status {
        int per_cu = 0;
        GP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0));
        per_cu = std::max(per_cu, 1);
        int64_t blocks = std::min<int64_t>(static_cast<int64_t>(per_cu) * sc->n_cu, sch.n_items);
        blocks = std::max<int64_t>(blocks, 1);
        gp_status r2 = grow(reinterpret_cast<void**>(&sc->tape), &sc->tape_cap,
                            static_cast<size_t>(blocks) * static_cast<size_t>(wave_floats), sizeof(float));
        if (r2 != GP_OK) return r2;
        hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(blocks)), dim3(kWave), 0, st, pv, cvw, dv, sch,
                           needs_forward ? sc->stats : nullptr, wsum, grad_fitness, lossp, sc->gpart, sc->gextra,
                           sc->tape, wave_floats);
        GP_HIP(hipGetLastError());
        return GP_OK;
    };
#define GP_ADJ_PICK(RR, F, M)                                                                  \
    (g_forced || occ(reinterpret_cast<const void*>(k_adjoint<RR, F, M>)) >=                    \
                     occ(reinterpret_cast<const void*>(k_adjoint<RR, 0, M>))                   \
         ? go(k_adjoint<RR, F, M>, adjoint_wave_floats<RR>(tape_max))                          \
         : go(k_adjoint<RR, 0, M>, adjoint_wave_floats<RR>(tape_max)))
#define GP_ADJ_R(RR, M)                                                                        \
    (freg == 2   ? GP_ADJ_PICK(RR, 2, M)                                                       \
     : freg == 8 ? GP_ADJ_PICK(RR, 8, M)                                                       \
                 : go(k_adjoint<RR, 0, M>, adjoint_wave_floats<RR>(tape_max)))
#define GP_ADJ_AUTO(M)                                                                         \
    (4 * occ(reinterpret_cast<const void*>(k_adjoint<4, 0, M>)) >                              \
             2 * occ(reinterpret_cast<const void*>(k_adjoint<2, 0, M>))                        \
         ? GP_ADJ_R(4, M)                                                                      \
         : GP_ADJ_R(2, M))
#define GP_ADJ(M) (RA == 0 ? GP_ADJ_AUTO(M) : RA == 1 ? GP_ADJ_R(1, M) : RA == 2 ? GP_ADJ_R(2, M) : GP_ADJ_R(4, M))
    switch (metric) {
    case GP_METRIC_MAE: rc = GP_ADJ(GP_METRIC_MAE); break;
    case GP_METRIC_MSE: rc = GP_ADJ(GP_METRIC_MSE); break;
    case GP_METRIC_RMSE: rc = GP_ADJ(GP_METRIC_RMSE); break;
    case GP_METRIC_LOGLOSS: rc = GP_ADJ(GP_METRIC_LOGLOSS); break;
    default: rc = GP_ADJ(GP_METRIC_PEARSON); break;
    }
#undef GP_ADJ
#undef GP_ADJ_AUTO
#undef GP_ADJ_R
#undef GP_ADJ_PICK
    if (rc != GP_OK) return rc;
    if (!needs_forward && fitness_out) {
        if (metric == GP_METRIC_MAE)
            hipLaunchKernelGGL(k_finalize<GP_METRIC_MAE>, dim3(fblocks), dim3(kBlock), 0, st, sc->part, sc->ystat,
                               sch.n_chunks, P, data->n_rows, has_w, fitness_out, nullptr);
        else if (metric == GP_METRIC_MSE)
            hipLaunchKernelGGL(k_finalize<GP_METRIC_MSE>, dim3(fblocks), dim3(kBlock), 0, st, sc->part, sc->ystat,
                               sch.n_chunks, P, data->n_rows, has_w, fitness_out, nullptr);
        else
            hipLaunchKernelGGL(k_finalize<GP_METRIC_LOGLOSS>, dim3(fblocks), dim3(kBlock), 0, st, sc->part,
                               sc->ystat, sch.n_chunks, P, data->n_rows, has_w, fitness_out, nullptr);
        GP_HIP(hipGetLastError());
    }
    if (pop->total_consts > 0) {
        hipLaunchKernelGGL(k_finalize_grad, dim3(fblocks), dim3(kBlock), 0, st, sc->gpart, sc->gextra,
                           pop->const_off, P, sch.n_chunks, grad_consts);
        GP_HIP(hipGetLastError());
    }
    return GP_OK;
}

}  // extern "C"
