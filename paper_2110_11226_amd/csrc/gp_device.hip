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
#include <mutex>
#include <string>
#include <vector>

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
    const uint2* code;
    const int32_t* clen;
};

// Work decomposition: rows are split into n_chunks chunks of `chunk` rows
// (a multiple of the 64*R rows one wavefront covers per tile).  Work item
// it = chunk_index * P + k covers program order[k] on that chunk; programs are
// ordered longest first so each chunk's long programs start early.
struct Sched {
    int64_t chunk;
    int32_t n_chunks;
    int64_t n_items;
    const int32_t* order;
    uint32_t* counter;
};

// ---------------------------------------------------------------------------
// Instruction format (word x; word y holds a constant's float bits):
//   bits 0-1  class: kPush (push a terminal), kFold (terminal fused with the
//             binary function whose first operand it is; the current top is
//             the second operand), kBin (binary: top op next-below), kUn
//   bits 2-4  function: binary ADD..DIV as 0..3, unary NEG..TAN as 0..5
//   bit 5     the terminal is a constant (value in y) rather than a feature
//   bits 8-31 feature index
// ---------------------------------------------------------------------------
enum : uint32_t { kPush = 0, kFold = 1, kBin = 2, kUn = 3 };

GP_HD uint32_t enc(uint32_t cls, uint32_t fn, uint32_t is_const, uint32_t arg) {
    return cls | (fn << 2) | (is_const << 5) | (arg << 8);
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

// Protected operators (reading of Sec. III-C3's function set: the gplearn
// convention).  Comparisons are written so that NaN takes the protected arm.
__device__ __forceinline__ float op_div(float a, float b) {
    return fabsf(b) > GP_PROTECT_EPS ? a / b : 1.0f;
}
__device__ __forceinline__ float op_log(float a) {
    return fabsf(a) > GP_PROTECT_EPS ? logf(fabsf(a)) : 0.0f;
}
__device__ __forceinline__ float op_sqrt(float a) { return sqrtf(fabsf(a)); }

// a = a (op) b for the binary function index fn (ADD, SUB, MUL, DIV)
template <int R>
__device__ __forceinline__ void apply_binary(uint32_t fn, float (&a)[R], const float (&b)[R]) {
    if (fn < 2) {
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

// t = f(t) for the unary function index fn (NEG, LOG, SQRT, SIN, COS, TAN)
template <int R>
__device__ __forceinline__ void apply_unary(uint32_t fn, float (&t)[R]) {
    if (fn < 3) {
        if (fn == 0) {
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = -t[j];
        } else if (fn == 1) {
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = op_log(t[j]);
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = op_sqrt(t[j]);
        }
    } else {
        if (fn == 3) {
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = sinf(t[j]);
        } else if (fn == 4) {
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = cosf(t[j]);
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
// such pairs become one kFold instruction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_compile(PopView pop, uint2* __restrict__ code,
                                                     int32_t* __restrict__ clen) {
    const int32_t p = static_cast<int32_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= pop.P) return;
    const int64_t off = pop.prog_off[p];
    const int32_t L = pop.len[p];
    const uint32_t* pn = pop.nodes + off;
    const float* pc = pop.consts + pop.const_off[p];
    uint2* out = code + off;
    int32_t k = 0;
    for (int32_t i = L - 1; i >= 0; --i) {
        const uint32_t w = pn[i];
        const uint32_t op = w & 0xffu;
        const uint32_t arg = w >> 8;
        if (op <= GP_OP_CONST) {
            const uint32_t is_c = op == GP_OP_CONST ? 1u : 0u;
            const uint32_t val = is_c ? __float_as_uint(pc[arg]) : 0u;
            const uint32_t farg = is_c ? 0u : arg;
            const uint32_t prev = i >= 1 ? (pn[i - 1] & 0xffu) : 0u;
            if (i >= 1 && i != L - 1 && prev >= GP_OP_ADD && prev <= GP_OP_DIV) {
                out[k++] = make_uint2(enc(kFold, prev - GP_OP_ADD, is_c, farg), val);
                --i;
            } else {
                out[k++] = make_uint2(enc(kPush, 0, is_c, farg), val);
            }
        } else if (op <= GP_OP_DIV) {
            out[k++] = make_uint2(enc(kBin, op - GP_OP_ADD, 0, 0), 0u);
        } else {
            out[k++] = make_uint2(enc(kUn, op - GP_OP_NEG, 0, 0), 0u);
        }
    }
    clen[p] = k;
}

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
        counter[0] = 0u;
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
    __shared__ float ovf_all[kBlock / kWave][kStackLds * R * kWave];
    float* ovf = ovf_all[threadIdx.x >> 6];

    for (;;) {
        uint32_t it32 = 0;
        if (lane == 0) it32 = atomicAdd(s.counter, 1u);
        const int64_t it = static_cast<int64_t>(__builtin_amdgcn_readlane(static_cast<int>(it32), 0));
        if (it >= s.n_items) break;   // every wavefront leaves here once the items run out
        const int32_t c = static_cast<int32_t>(it / pop.P);
        const int32_t k = static_cast<int32_t>(it - static_cast<int64_t>(c) * pop.P);
        const int32_t p = ldu(s.order + k);
        const int64_t off = ldu(pop.prog_off + p);
        const int32_t CL = ldu(cv.clen + p);
        const uint2* __restrict__ pcode = cv.code + off;
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

            // ---- the stack machine (Sec. III-A order, compiled by k_compile) ----
            // t[] is the top of the stack; slot `dp` (VGPRs below kStackRegs,
            // LDS from there on) is the entry just below it.  Every instruction
            // first writes the top into the slot above dp -- kept only when the
            // instruction is a push, which then just advances dp -- so the
            // register array sees exactly one indexed write per instruction and
            // is never copied.  The first push parks the empty top in slot 0,
            // which is never read back.  The next instruction is fetched one
            // step ahead as a vector register and made scalar where it is used.
            float t[R];
#pragma unroll
            for (int j = 0; j < R; ++j) t[j] = 0.0f;
            GP_ARRAYS(st, kStackRegs + 1);
            int dp = -1;
            uint2 nxt = pcode[0];
            for (int q = 0; q < CL; ++q) {
                const uint2 cur = nxt;
                nxt = pcode[min(q + 1, CL - 1)];
                const uint32_t w = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(cur.x)));
                const uint32_t cls = w & 3u;
                const uint32_t fn = (w >> 2) & 7u;
                const int up = min(dp + 1, kStackRegs);
                GP_PUT(st, up, t);
                if (cls == kUn) {
                    apply_unary<R>(fn, t);
                    continue;
                }
                float a[R], b[R];
                if (cls == kBin) {
                    if (dp < kStackRegs) {
                        GP_GET(st, dp, b);
                    } else {
#pragma unroll
                        for (int j = 0; j < R; ++j) b[j] = ovf[((dp - kStackRegs) * R + j) * kWave + lane];
                    }
                    --dp;
#pragma unroll
                    for (int j = 0; j < R; ++j) a[j] = t[j];
                } else {
                    float v[R];
                    if (w & 32u) {
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
                        continue;
                    }
                    // kFold: the terminal is the first operand, the top the second
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        a[j] = v[j];
                        b[j] = t[j];
                    }
                }
                apply_binary<R>(fn, a, b);
#pragma unroll
                for (int j = 0; j < R; ++j) t[j] = a[j];
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

template <int METRIC>
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ part,
                                                      const double* __restrict__ ystat,
                                                      int32_t n_chunks, int32_t P, int64_t N,
                                                      int has_w, float* __restrict__ fitness) {
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
            if (va > 0.0 && vb > 0.0 && isfinite(va) && isfinite(vb)) r = fabs(m.Mab / sqrt(va * vb));
            fitness[p] = static_cast<float>(r);
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
        }
    }
}

// ---------------------------------------------------------------------------
// k_tournament (Sec. III-C1): one lane per tournament.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_tournament(const float* __restrict__ fit,
                                                        const int32_t* __restrict__ len,
                                                        int32_t P, int larger, float c, int32_t k,
                                                        int32_t T, uint64_t seed, uint32_t gen,
                                                        int32_t* __restrict__ winners) {
    const int32_t t = static_cast<int32_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= T) return;
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
// Host side: scratch, launch configuration, entry points.
// ---------------------------------------------------------------------------
#define GP_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(GP_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

struct DeviceScratch {
    void* counter = nullptr;     // 256 bytes: the work counter
    int32_t* order = nullptr;
    size_t order_cap = 0;
    double* part = nullptr;
    size_t part_cap = 0;         // doubles
    double* ystat = nullptr;
    size_t ystat_cap = 0;        // doubles
    uint2* code = nullptr;
    size_t code_cap = 0;         // instructions
    int32_t* clen = nullptr;
    size_t clen_cap = 0;
    int n_cu = 0;
};

std::mutex g_mu;
std::vector<DeviceScratch> g_dev;

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

gp_status scratch_for(int dev, DeviceScratch** out) {
    if (static_cast<int>(g_dev.size()) <= dev) g_dev.resize(dev + 1);
    DeviceScratch& s = g_dev[dev];
    if (!s.counter) {
        GP_HIP(hipMalloc(&s.counter, 256));
        GP_HIP(hipMemset(s.counter, 0, 256));
        hipDeviceProp_t prop;
        GP_HIP(hipGetDeviceProperties(&prop, dev));
        s.n_cu = prop.multiProcessorCount;
    }
    *out = &s;
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

// Launch configuration of the evaluation kernel.
struct LaunchCfg {
    int R;        // rows per lane: 1, 2 or 4
    int freg;     // features held in registers: 0, 2 or 8
    int tiles;    // tiles of 64*R rows per chunk
};

bool g_forced = false;
LaunchCfg g_forced_cfg{4, 0, 1};

LaunchCfg pick_cfg(int F, int64_t N, int32_t P, int n_cu) {
    if (g_forced) return g_forced_cfg;
    LaunchCfg c;
    c.R = 4;
    c.freg = F <= 2 ? 2 : (F <= 8 ? 8 : 0);
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

template <int MODE, int METRIC>
gp_status launch_eval_m(const LaunchCfg& cfg, int n_cu, const PopView& pv, const CodeView& cv,
                        const DataView& dv, const Sched& s, float* out, double* part, hipStream_t st,
                        int64_t node_rows) {
    auto go = [&](auto kernel) -> gp_status {
        int per_cu = 0;
        GP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0));
        per_cu = std::max(per_cu, 1);
        const int64_t waves_needed = s.n_items;
        int64_t blocks = static_cast<int64_t>(per_cu) * n_cu;
        blocks = std::min<int64_t>(blocks, (waves_needed + (kBlock / kWave) - 1) / (kBlock / kWave));
        blocks = std::max<int64_t>(blocks, 1);
        ProfRec rec{nullptr, nullptr, node_rows};
        if (g_prof_on) {
            GP_HIP(hipEventCreate(&rec.a));
            GP_HIP(hipEventCreate(&rec.b));
            GP_HIP(hipEventRecord(rec.a, st));
        }
        hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, st, pv, cv, dv, s, out,
                           part);
        GP_HIP(hipGetLastError());
        if (g_prof_on) {
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
                      hipStream_t st, int64_t node_rows) {
    if (mode == 0)
        return launch_eval_m<0, GP_METRIC_MSE>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows);
    switch (metric) {
    case GP_METRIC_MAE:
        return launch_eval_m<1, GP_METRIC_MAE>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows);
    case GP_METRIC_MSE:
    case GP_METRIC_RMSE:
        return launch_eval_m<1, GP_METRIC_MSE>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows);
    case GP_METRIC_LOGLOSS:
        return launch_eval_m<1, GP_METRIC_LOGLOSS>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows);
    case GP_METRIC_PEARSON:
        return launch_eval_m<1, GP_METRIC_PEARSON>(cfg, n_cu, pv, cv, dv, s, out, part, st, node_rows);
    default: return fail(GP_ERR_UNSUPPORTED, "metric not supported by the fused fitness kernel");
    }
}

// Shared front half of gp_evaluate / gp_fitness: checks, scratch, ordering.
gp_status prepare(const gp_population_dev* pop, const gp_dataset_dev* data, int mode, int metric,
                  hipStream_t st, DeviceScratch** sc_out, PopView* pv, CodeView* cvw, DataView* dv,
                  Sched* sch, LaunchCfg* cfg) {
    int dev = 0;
    GP_HIP(hipGetDevice(&dev));
    DeviceScratch* sc = nullptr;
    gp_status rc = scratch_for(dev, &sc);
    if (rc != GP_OK) return rc;
    *pv = PopView{pop->nodes, pop->prog_off, pop->consts, pop->const_off, pop->len, pop->n_programs};
    *dv = DataView{data->X, data->ld, data->n_features, data->n_rows, data->y, data->w};
    *cfg = pick_cfg(data->n_features, data->n_rows, pop->n_programs, sc->n_cu);
    if (cfg->freg > 0 && data->n_features > cfg->freg)
        return fail(GP_ERR_INVALID_ARG, "launch configuration holds fewer feature registers than n_features");
    const int64_t chunk = static_cast<int64_t>(cfg->tiles) * kWave * cfg->R;
    const int64_t n_chunks = (data->n_rows + chunk - 1) / chunk;
    const int64_t n_items = n_chunks * pop->n_programs;
    // the 32-bit work counter overshoots n_items by at most one per wavefront
    if (n_items > (int64_t{1} << 30))
        return fail(GP_ERR_INVALID_ARG, "too many work items (n_programs * row chunks above 2^30)");
    rc = grow(reinterpret_cast<void**>(&sc->order), &sc->order_cap, pop->n_programs, sizeof(int32_t));
    if (rc != GP_OK) return rc;
    rc = grow(reinterpret_cast<void**>(&sc->code), &sc->code_cap, static_cast<size_t>(pop->total_nodes),
              sizeof(uint2));
    if (rc != GP_OK) return rc;
    rc = grow(reinterpret_cast<void**>(&sc->clen), &sc->clen_cap, pop->n_programs, sizeof(int32_t));
    if (rc != GP_OK) return rc;
    if (mode == 1) {
        const size_t kk = metric == GP_METRIC_PEARSON ? 4 : 1;
        rc = grow(reinterpret_cast<void**>(&sc->part), &sc->part_cap,
                  static_cast<size_t>(pop->n_programs) * n_chunks * kk, sizeof(double));
        if (rc != GP_OK) return rc;
        rc = grow(reinterpret_cast<void**>(&sc->ystat), &sc->ystat_cap, static_cast<size_t>(n_chunks) * 4,
                  sizeof(double));
        if (rc != GP_OK) return rc;
    }
    *sch = Sched{chunk, static_cast<int32_t>(n_chunks), n_items, sc->order,
                 static_cast<uint32_t*>(sc->counter)};
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(1024), 0, st, pop->len, pop->n_programs, sc->order,
                       static_cast<uint32_t*>(sc->counter));
    GP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_compile, dim3((pop->n_programs + kBlock - 1) / kBlock), dim3(kBlock), 0, st, *pv,
                       sc->code, sc->clen);
    GP_HIP(hipGetLastError());
    *cvw = CodeView{sc->code, sc->clen};
    *sc_out = sc;
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
        if (!s.counter && !s.order && !s.part && !s.ystat && !s.code && !s.clen) continue;
        (void)hipSetDevice(static_cast<int>(d));
        (void)hipDeviceSynchronize();
        if (s.counter) (void)hipFree(s.counter);
        if (s.order) (void)hipFree(s.order);
        if (s.part) (void)hipFree(s.part);
        if (s.ystat) (void)hipFree(s.ystat);
        if (s.code) (void)hipFree(s.code);
        if (s.clen) (void)hipFree(s.clen);
        s = DeviceScratch{};
    }
    (void)hipSetDevice(cur);
}

gp_status gp_get_launch_config(int32_t n_features, int64_t n_rows, int32_t n_programs,
                               gp_launch_config* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!out || n_features < 1 || n_rows < 1 || n_programs < 0)
        return fail(GP_ERR_INVALID_ARG, "gp_get_launch_config: bad arguments");
    int dev = 0;
    GP_HIP(hipGetDevice(&dev));
    DeviceScratch* sc = nullptr;
    gp_status rc = scratch_for(dev, &sc);
    if (rc != GP_OK) return rc;
    const LaunchCfg c = pick_cfg(n_features, n_rows, n_programs, sc->n_cu);
    *out = gp_launch_config{c.R, c.freg, c.tiles};
    return GP_OK;
}

gp_status gp_set_launch_config(const gp_launch_config* cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!cfg) {
        g_forced = false;
        return GP_OK;
    }
    const bool r_ok = cfg->rows_per_lane == 1 || cfg->rows_per_lane == 2 || cfg->rows_per_lane == 4;
    const bool f_ok = cfg->feature_regs == 0 || cfg->feature_regs == 2 || cfg->feature_regs == 8;
    if (!r_ok || !f_ok || cfg->tiles_per_chunk < 1 || cfg->tiles_per_chunk > (1 << 20))
        return fail(GP_ERR_INVALID_ARG, "gp_set_launch_config: rows_per_lane in {1,2,4}, feature_regs in {0,2,8}, "
                                        "tiles_per_chunk in [1, 2^20]");
    g_forced_cfg = LaunchCfg{cfg->rows_per_lane, cfg->feature_regs, cfg->tiles_per_chunk};
    g_forced = true;
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
    PopView pv;
    CodeView cvw;
    DataView dv;
    Sched sch;
    LaunchCfg cfg;
    rc = prepare(pop, data, 0, GP_METRIC_MSE, st, &sc, &pv, &cvw, &dv, &sch, &cfg);
    if (rc != GP_OK) return rc;
    return launch_eval(0, GP_METRIC_MSE, cfg, sc->n_cu, pv, cvw, dv, sch, out, nullptr, st,
                       pop->total_nodes * data->n_rows);
}

gp_status gp_fitness(const gp_population_dev* pop, const gp_dataset_dev* data, gp_metric metric,
                     float* fitness, void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    gp_status rc = check_pop(pop, "gp_fitness");
    if (rc != GP_OK) return rc;
    rc = check_data(data, "gp_fitness", true);
    if (rc != GP_OK) return rc;
    if (!fitness) return fail(GP_ERR_INVALID_ARG, "gp_fitness: fitness is NULL");
    if (metric == GP_METRIC_SPEARMAN)
        return fail(GP_ERR_UNSUPPORTED, "gp_fitness: Spearman is not provided by this version");
    if (gp_metric_larger_is_better(metric) < 0) return fail(GP_ERR_INVALID_ARG, "gp_fitness: unknown metric");
    if (pop->n_programs == 0) return GP_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DeviceScratch* sc;
    PopView pv;
    CodeView cvw;
    DataView dv;
    Sched sch;
    LaunchCfg cfg;
    rc = prepare(pop, data, 1, metric, st, &sc, &pv, &cvw, &dv, &sch, &cfg);
    if (rc != GP_OK) return rc;
    const bool need_ystats = data->w != nullptr || metric == GP_METRIC_PEARSON;
    if (need_ystats) {
        const int blocks = (sch.n_chunks + (kBlock / kWave) - 1) / (kBlock / kWave);
        hipLaunchKernelGGL(k_ystats, dim3(blocks), dim3(kBlock), 0, st, dv, sch.chunk, sch.n_chunks, sc->ystat);
        GP_HIP(hipGetLastError());
    }
    rc = launch_eval(1, metric, cfg, sc->n_cu, pv, cvw, dv, sch, nullptr, sc->part, st,
                     pop->total_nodes * data->n_rows);
    if (rc != GP_OK) return rc;
    const int fblocks = (pop->n_programs + (kBlock / kWave) - 1) / (kBlock / kWave);
    const int has_w = data->w != nullptr;
#define GP_FIN(M)                                                                                  \
    hipLaunchKernelGGL(k_finalize<M>, dim3(fblocks), dim3(kBlock), 0, st, sc->part, sc->ystat,   \
                       sch.n_chunks, pop->n_programs, data->n_rows, has_w, fitness)
    switch (metric) {
    case GP_METRIC_MAE: GP_FIN(GP_METRIC_MAE); break;
    case GP_METRIC_MSE: GP_FIN(GP_METRIC_MSE); break;
    case GP_METRIC_RMSE: GP_FIN(GP_METRIC_RMSE); break;
    case GP_METRIC_LOGLOSS: GP_FIN(GP_METRIC_LOGLOSS); break;
    default: GP_FIN(GP_METRIC_PEARSON); break;
    }
#undef GP_FIN
    GP_HIP(hipGetLastError());
    return GP_OK;
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
    const int blocks = (n_tournaments + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_tournament, dim3(blocks), dim3(kBlock), 0, static_cast<hipStream_t>(stream), fitness,
                       len, n_programs, larger, parsimony, tournament_size, n_tournaments, seed,
                       static_cast<uint32_t>(generation), winners);
    GP_HIP(hipGetLastError());
    return GP_OK;
}

gp_status gp_fitness_backward(const gp_population_dev* pop, const gp_dataset_dev* data, gp_metric metric,
                              const float* grad_fitness, float* fitness_out, float* grad_consts,
                              void* stream) {
    (void)pop; (void)data; (void)metric; (void)grad_fitness; (void)fitness_out; (void)grad_consts;
    (void)stream;
    return fail(GP_ERR_UNSUPPORTED, "gp_fitness_backward: not built yet");
}

}  // extern "C"
