/*
 * gp.h -- C ABI of the MI355X (gfx950) GP population-evaluation library.
 *
 * The library implements the data-parallel hot path of stack-based
 * generational genetic programming as described in "Accelerating Genetic
 * Programming using GPUs" (arXiv 2110.11226): evaluate every program of a
 * population of prefix lists on every row of a dataset resident in device
 * memory (Sec. III intro, Sec. III-C3 execution step), reduce each program's
 * row losses to its fitness (Sec. III-C3, fitness metric computation step) and
 * select parents by tournament with a parsimony penalty (Sec. III-C1).  It
 * also generates initial populations (Sec. II-A) and, beyond the paper, gives
 * the derivative of fitness with respect to every program constant.
 *
 * Conventions for every entry point:
 *   - Plain C types only.  Pointers documented "device" must point to device
 *     memory on the current HIP device; "host" pointers to host memory.
 *   - Device entry points are asynchronous on `stream` (a hipStream_t passed
 *     as void*, NULL = the null stream).  Arguments are checked on the host
 *     before anything is launched; a non-OK status means nothing was
 *     launched.  Faults inside kernels surface as GP_ERR_DEVICE on a later
 *     call or at the caller's synchronisation.
 *   - The caller owns every buffer it passes.  Scratch space (partial sums,
 *     work counters, orderings) is owned by the library, kept per device and
 *     grown on demand; gp_shutdown() releases it.  Calls that share a device
 *     share this scratch: issue them on one stream (or serialise them).
 *   - No C++ exception crosses this boundary.  On failure the status is
 *     returned and gp_last_error() holds a thread-local description.
 */
#ifndef GP_H
#define GP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ */
/* Program encoding (Sec. III-A: a program is its expression tree in   */
/* Polish (prefix) order; functions have arity at most 2, Sec. III).   */
/* A node is one uint32: opcode in bits 0-7, argument in bits 8-31.    */
/* GP_OP_VAR's argument is a feature index; GP_OP_CONST's argument is  */
/* a slot in the program's own constant table.                         */
/* ------------------------------------------------------------------ */
enum {
    GP_OP_VAR = 0,   /* terminal: feature value X[arg][row]                       */
    GP_OP_CONST = 1, /* terminal: constant consts[const_off[p] + arg]             */
    GP_OP_ADD = 2,   /* a + b                                                      */
    GP_OP_SUB = 3,   /* a - b   (a is the first argument, b the second)           */
    GP_OP_MUL = 4,   /* a * b                                                      */
    GP_OP_DIV = 5,   /* protected: |b| > 0.001f ? a / b : 1                        */
    GP_OP_NEG = 6,   /* -a                                                         */
    GP_OP_LOG = 7,   /* protected: |a| > 0.001f ? log|a| : 0                       */
    GP_OP_SQRT = 8,  /* protected: sqrt|a|                                         */
    GP_OP_SIN = 9,   /* sin a                                                      */
    GP_OP_COS = 10,  /* cos a                                                      */
    GP_OP_TAN = 11,  /* tan a                                                      */
    /* the wider set (the paper counts its functions without listing them) */
    GP_OP_MAX = 12,   /* IEEE 754-2019 maximumNumber: a NaN operand yields the    */
                      /* other; -0 orders below +0                                */
    GP_OP_MIN = 13,   /* minimumNumber: a NaN operand yields the other; -0 < +0   */
    GP_OP_ATAN2 = 14, /* atan2f(a, b): a is y, b is x                             */
    GP_OP_ABS = 15,   /* |a|                                                      */
    GP_OP_EXP = 16,   /* exp a                                                    */
    GP_OP_INV = 17,   /* protected: |a| > 0.001f ? 1 / a : 0                      */
    GP_OP_SQ = 18,    /* a * a                                                    */
    GP_OP_CUBE = 19,  /* (a * a) * a                                              */
    GP_OP_TANH = 20,  /* tanh a                                                   */
    GP_OP_ATAN = 21,  /* atan a                                                   */
    GP_OP_CBRT = 22,  /* cube root of a                                           */
    GP_OP_COUNT = 23,
    /* user-defined functions (Sec. V: custom function sets), registered with
     * gp_register_function: 24..27 take one argument, 28..31 two */
    GP_OP_USER1 = 24,
    GP_OP_USER2 = 28,
    GP_OP_LIMIT = 32  /* every opcode is below this                             */
};
#define GP_NODE(op, arg) ((uint32_t)(op) | ((uint32_t)(arg) << 8))
#define GP_NODE_OP(w) ((uint32_t)(w) & 0xffu)
#define GP_NODE_ARG(w) ((uint32_t)(w) >> 8)

/* Evaluation stack depth (Sec. III-B fixed-size device stack; the paper's
 * stack of m slots evaluates trees of depth m-1, Sec. III-C2).  A program is
 * valid iff its right-to-left stack height never exceeds this. */
#define GP_MAX_STACK 20
/* Threshold of the protected operators (the float nearest 0.001). */
#define GP_PROTECT_EPS 0.001f
/* The nine-function set {add, sub, mul, div, neg, log, sqrt, sin, cos}. */
#define GP_FUNCS_DEFAULT 0x7FCu

/* ------------------------------------------------------------------ */
/* Status                                                              */
/* ------------------------------------------------------------------ */
typedef enum {
    GP_OK = 0,
    GP_ERR_INVALID_ARG = -1,      /* a null pointer, a size out of range, ...      */
    GP_ERR_INVALID_PROGRAM = -2,  /* bad opcode / feature / constant slot / arity  */
    GP_ERR_STACK_OVERFLOW = -3,   /* stack height above GP_MAX_STACK               */
    GP_ERR_OUT_OF_MEMORY = -4,    /* scratch allocation failed                     */
    GP_ERR_DEVICE = -5,           /* a HIP runtime error                           */
    GP_ERR_UNSUPPORTED = -6,      /* e.g. a metric this entry point does not have  */
    GP_ERR_BUFFER_TOO_SMALL = -7  /* a caller buffer below the size it needs       */
} gp_status;

/* Thread-local text for the last non-OK status returned on this thread. */
const char* gp_last_error(void);
/* Library version string. */
const char* gp_version(void);
/* Release the per-device scratch of every device.  Safe to call twice. */
void gp_shutdown(void);

/* ------------------------------------------------------------------ */
/* Fitness metrics (Sec. III-C3: weighted MAE, MSE, RMSE, logistic     */
/* loss, Pearson and Spearman correlation).  Weights w == NULL mean 1. */
/*   MAE  = sum w|yh-y| / sum w           (smaller is better)          */
/*   MSE  = sum w(yh-y)^2 / sum w         (smaller is better)          */
/*   RMSE = sqrt(MSE)                     (smaller is better)          */
/*   LOGLOSS: yh is a logit, row loss max(yh,0) - y yh + log1p(e^-|yh|)*/
/*            with y in {0,1}, weighted mean (smaller is better)       */
/*   PEARSON: |weighted correlation of yh and y|, 0 when a variance is */
/*            zero or not finite (larger is better)                    */
/*   SPEARMAN: |weighted correlation of the ranks of yh and of y|:     */
/*            rank 1 the smallest, tied values the mean of their       */
/*            ranks, ranks unweighted, the weights in the correlation; */
/*            0 for a constant rank vector, NaN if any yh or y is NaN  */
/*            (larger is better).  gp_fitness, the generation graphs   */
/*            and the evolution loop compute it (batched sort on the   */
/*            device, n_rows below 2^31); gp_fitness_backward,         */
/*            gp_autotune and gp_get_launch_config give                */
/*            GP_ERR_UNSUPPORTED (ranks have no derivative).           */
/* Row losses of MAE/MSE/RMSE/PEARSON are formed in float64 from the   */
/* float32 program value; LOGLOSS's in float32; all row sums in        */
/* float64; the result is rounded to float32.                          */
/* ------------------------------------------------------------------ */
/*   USER_0..USER_3 (Sec. V: custom loss functions): the row loss is the */
/*            float32 value of the registered two-argument user function */
/*            GP_OP_USER2 + i applied to (yh, y); fitness = sum w l /    */
/*            sum w in float64 (smaller is better).  gp_fitness and the  */
/*            generation graphs and evolution loop compute it;           */
/*            gp_fitness_backward gives GP_ERR_UNSUPPORTED.              */
typedef enum {
    GP_METRIC_MAE = 0,
    GP_METRIC_MSE = 1,
    GP_METRIC_RMSE = 2,
    GP_METRIC_LOGLOSS = 3,
    GP_METRIC_PEARSON = 4,
    GP_METRIC_SPEARMAN = 5,
    GP_METRIC_USER_0 = 6,
    GP_METRIC_USER_1 = 7,
    GP_METRIC_USER_2 = 8,
    GP_METRIC_USER_3 = 9
} gp_metric;

/* ------------------------------------------------------------------ */
/* User-defined functions (Sec. V: custom function sets and loss      */
/* functions during GP runs).                                          */
/* ------------------------------------------------------------------ */
/* Maximum size of a definition and the stack it may use on its own. */
#define GP_USER_MAX_NODES 32
#define GP_USER_MAX_CONSTS 16
#define GP_USER_MAX_STACK 6

/* Define user function `op` (GP_OP_USER1 .. GP_OP_USER1+3: one argument;
 * GP_OP_USER2 .. GP_OP_USER2+3: two) as an expression over the built-in
 * functions: def[def_len] is a prefix list (the program encoding above) in
 * which GP_NODE(GP_OP_VAR, k) stands for argument k (k < the function's
 * arity; argument 0 is the first) and GP_NODE(GP_OP_CONST, k) for
 * consts[k].  A program node `op` then evaluates to the definition's value
 * on its arguments, every operation rounded to float32 as when the
 * definition is written out in the program.  The definition may not use
 * user functions, must leave exactly one value and may hold at most
 * GP_USER_MAX_STACK values on the right-to-left scan (this stack comes on
 * top of the program's GP_MAX_STACK).  def_len == 0 removes the definition.
 * Once defined, `op` may appear in programs (gp_validate_population accepts
 * it), in function_mask (bit 1 << op) of the generators and mutation, and a
 * two-argument function may serve as the row loss of GP_METRIC_USER_i
 * (op = GP_OP_USER2 + i).  Process-wide; it applies to calls made after it
 * and to generation graphs and evolution loops created after it (those
 * created before keep what they captured).  Not thread-safe against
 * concurrent evaluation calls.  gp_fitness_backward gives
 * GP_ERR_UNSUPPORTED for populations that use user functions. */
gp_status gp_register_function(uint32_t op, const uint32_t* def, int32_t def_len, const float* consts,
                               int32_t n_consts);
/* 1 if user function op is defined, else 0. */
int gp_function_defined(uint32_t op);

/* 1 if a larger value of the metric is better (Sec. III-C1: the criterion
 * may favour smaller or larger values), 0 if smaller is better, -1 if the
 * metric is unknown. */
int gp_metric_larger_is_better(gp_metric metric);

/* ------------------------------------------------------------------ */
/* Population generation (Sec. II-A: Full, Grow, ramped half-and-half; */
/* prefix lists are generated directly, Sec. III-A), plus an exact-    */
/* length generator.  Host-only.  Draws come from Philox4x32-10        */
/* (Sec. III-B) with key = seed and counter = (block, program index,   */
/* 0, 1); one 32-bit word per decision, taken in prefix order:         */
/*  RHH: Grow if unit(word) < 0.5 else Full; depth in                  */
/*   [min_depth, max_depth].  Node at depth k of a tree of depth d:    */
/*   k == d -> terminal; k == 0 < d -> function; otherwise Full ->     */
/*   function, Grow -> uniform over (functions, features, constant).   */
/*  EXACT_LEN: length in [min_len, max_len]; positions filled right to */
/*   left under the stack-height rule so the program is valid; uniform */
/*   over the allowed (features, constant, unary ops, binary ops).     */
/* A constant is const_lo + (const_hi - const_lo) * unit(word) in      */
/* float32.  Constants are off when const_lo > const_hi or once        */
/* max_consts (> 0) are used.  unit(word) = (word >> 8) * 2^-24;       */
/* a choice among n uses floor(word * n / 2^32).  Constant slots are   */
/* numbered 0, 1, ... in prefix order.                                 */
/* ------------------------------------------------------------------ */
typedef enum {
    GP_INIT_RHH = 0,
    GP_INIT_FULL = 1,
    GP_INIT_GROW = 2,
    GP_INIT_EXACT_LEN = 3
} gp_init;

typedef struct {
    int32_t n_programs;       /* >= 0                                             */
    int32_t n_features;       /* >= 1                                             */
    int32_t method;           /* gp_init                                          */
    int32_t min_depth;        /* RHH / FULL / GROW: 0 <= min <= max <= 19          */
    int32_t max_depth;
    int32_t min_len;          /* EXACT_LEN: 1 <= min <= max <= 1<<20               */
    int32_t max_len;
    uint32_t function_mask;   /* bit (1 << opcode) for each enabled function      */
    float const_lo;           /* constants ~ U[lo, hi); lo > hi disables them      */
    float const_hi;
    int32_t max_consts;       /* 0 = unlimited                                     */
    uint64_t seed;
} gp_init_params;

/* Generate a population into caller-owned HOST buffers.
 * Two-call idiom: with nodes == NULL only *total_nodes / *total_consts are
 * written.  Otherwise nodes[nodes_cap], prog_off[n_programs+1],
 * consts[consts_cap], const_off[n_programs+1] and len[n_programs] receive the
 * flat population; GP_ERR_BUFFER_TOO_SMALL if a capacity is short. */
gp_status gp_build_population(const gp_init_params* params,
                              uint32_t* nodes, int64_t nodes_cap, int64_t* prog_off,
                              float* consts, int64_t consts_cap, int64_t* const_off,
                              int32_t* len, int64_t* total_nodes, int64_t* total_consts);

/* Check a HOST population: every opcode known, every feature index below
 * n_features, every constant slot below that program's constant count,
 * exactly one value left and stack height <= GP_MAX_STACK on the
 * right-to-left scan (Sec. III-A, III-C2).  max_height[n_programs]
 * (nullable) receives each program's peak stack height.  On failure
 * *bad_program (nullable) receives the first offending program. */
gp_status gp_validate_population(const uint32_t* nodes, const int64_t* prog_off,
                                 const int64_t* const_off, int32_t n_programs,
                                 int32_t n_features, int32_t* max_height,
                                 int32_t* bad_program);

/* ------------------------------------------------------------------ */
/* Genetic operations on the host (Sec. II-A mutation list; Sec. III-C */
/* pre-draw of operation types; Sec. III-C2 hoisted crossover).  Draws */
/* come from Philox4x32-10 with key seed and counter (block, offspring */
/* i, generation, 2), consumed in order; donor programs of subtree     */
/* mutation from counter (block, i, generation, 3).                    */
/* ------------------------------------------------------------------ */
typedef enum {
    GP_GENOP_CROSSOVER = 0,     /* 2 tournaments: parent, donor                    */
    GP_GENOP_SUBTREE = 1,       /* crossover with a freshly generated donor        */
    GP_GENOP_HOIST = 2,
    GP_GENOP_POINT = 3,
    GP_GENOP_REPRODUCTION = 4
} gp_genetic_op;

typedef struct {
    float p_crossover;        /* operation probabilities, each in [0, 1]; the     */
    float p_subtree;          /* float32 running sums crossover, subtree, hoist,  */
    float p_hoist;            /* point must stay <= 1; reproduction takes the     */
    float p_point;            /* rest                                              */
    float p_point_replace;    /* per-node replacement probability (point)          */
    int32_t max_len;          /* length bound of crossover children (>= 1)         */
    uint64_t seed;
} gp_evolve_params;

/* The operation of every offspring (draw 0 of its stream: the first k with
 * u < running sum k, else reproduction) and where its tournaments start in
 * the winners array: first_tournament is the prefix sum of the tournaments
 * each operation needs (crossover 2, others 1), *n_tournaments the total.
 * ops and first_tournament are HOST arrays [n_offspring]. */
gp_status gp_plan_generation(const gp_evolve_params* params, int32_t n_offspring, uint64_t generation,
                             int32_t* ops, int32_t* first_tournament, int32_t* n_tournaments);

/* Offspring i from parent winners[first_tournament[i]] (and, for crossover,
 * donor winners[first_tournament[i] + 1]) of the HOST parent population:
 *   crossover: a uniformly chosen subtree of the parent is replaced by a
 *     uniformly chosen subtree of the donor (draws 1, 2); while the child's
 *     stack height exceeds GP_MAX_STACK or its length max_len, the donor
 *     subtree is replaced by a uniformly chosen proper subtree of itself (one
 *     draw each) -- the hoisted crossover;
 *   subtree: the same with a donor program generated by `init`'s method,
 *     function set, depths or lengths and constants;
 *   hoist: a uniformly chosen subtree is replaced by a uniformly chosen
 *     subtree of itself (draws 1, 2);
 *   point: each node in prefix order is replaced when its draw u <
 *     p_point_replace: a function by one of the same arity (one draw), a
 *     terminal by a variable or a new constant (one draw, and one for the
 *     value; constants only while the program's others number below
 *     init->max_consts);
 *   reproduction: a copy.
 * "Uniformly chosen subtree" means a uniformly chosen node position.
 * Constants keep their values and are renumbered in prefix order.  Parents
 * are validated first.  The offspring population goes to caller-owned HOST
 * buffers with capacities nodes_cap / consts_cap (GP_ERR_BUFFER_TOO_SMALL
 * with *total_nodes / *total_consts set if short); out_prog_off and
 * out_const_off [n_offspring + 1], out_len [n_offspring]. */
gp_status gp_mutate(const gp_evolve_params* params, const gp_init_params* init,
                    const uint32_t* nodes, const int64_t* prog_off, const float* consts,
                    const int64_t* const_off, int32_t n_parents, const int32_t* ops,
                    const int32_t* first_tournament, const int32_t* winners, int32_t n_winners,
                    int32_t n_offspring, uint64_t generation, uint32_t* out_nodes, int64_t nodes_cap,
                    int64_t* out_prog_off, float* out_consts, int64_t consts_cap,
                    int64_t* out_const_off, int32_t* out_len, int64_t* total_nodes,
                    int64_t* total_consts);

/* ------------------------------------------------------------------ */
/* Device views                                                        */
/* ------------------------------------------------------------------ */
/* A flat population in DEVICE memory (Sec. III-A program struct, laid out
 * as one structure of arrays instead of the paper's array of structs with
 * nested pointers, Sec. III-D2).  Program p is nodes[prog_off[p] ..
 * prog_off[p]+len[p]) with constants consts[const_off[p] ..).  Programs must
 * be valid (gp_validate_population); device code does not re-check. */
typedef struct {
    const uint32_t* nodes;
    const int64_t* prog_off;   /* [n_programs + 1] */
    const float* consts;
    const int64_t* const_off;  /* [n_programs + 1] */
    const int32_t* len;        /* [n_programs], len[p] = prog_off[p+1]-prog_off[p] */
    int32_t n_programs;
    int64_t total_nodes;
    int32_t max_len;           /* an upper bound on every len[p] (host-known)   */
    int64_t total_consts;      /* const_off[n_programs] (host-known)            */
} gp_population_dev;

/* A dataset in DEVICE memory, feature-major (the paper's column-major
 * layout, Sec. III intro): feature f of row r is X[f * ld + r]. */
typedef struct {
    const float* X;
    int64_t ld;                /* >= n_rows */
    int32_t n_features;
    int64_t n_rows;            /* >= 1 */
    const float* y;            /* [n_rows] target / binary label */
    const float* w;            /* [n_rows] sample weights, or NULL for 1 */
} gp_dataset_dev;

/* ------------------------------------------------------------------ */
/* Hot path                                                            */
/* ------------------------------------------------------------------ */
/* Program outputs (Sec. III-C3 execution step): out[p * n_rows + r] =
 * float32 value of program p on row r (right-to-left stack evaluation,
 * Sec. III-A).  out is DEVICE memory of n_programs * n_rows floats. */
gp_status gp_evaluate(const gp_population_dev* pop, const gp_dataset_dev* data,
                      float* out, void* stream);

/* Fitness of every program (Sec. III-C3: execution, row loss against the
 * broadcast target, weighted reduction per program), fused so that per-row
 * outputs never reach memory.  fitness is DEVICE memory [n_programs]. */
gp_status gp_fitness(const gp_population_dev* pop, const gp_dataset_dev* data,
                     gp_metric metric, float* fitness, void* stream);

/* gp_fitness for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, launch configuration and result as gp_fitness, with the
 * scratch (work counter, length order, instruction stream, per-chunk
 * partial sums) taken from a static 64 MiB device array that the library
 * holds on every device it runs on until the process ends.  It allocates
 * nothing on the device (no hipMalloc, hipFree or allocating library call)
 * and needs
 *   1024 + 2 a(4 P) + a(16 (total_nodes m + P u + 1)) + a(8 P C k) + a(32 C)
 * bytes, a(n) = n rounded up to 256, C = the launch's row chunks
 * (ceil(n_rows / (tiles_per_chunk * 64 * rows_per_lane)), gp_get_launch_config),
 * k = 4 for PEARSON else 1, m = 1 (or, while user functions are defined,
 * the longest definition's length), u = 0 (for a user loss, 1 + its
 * definition's length); above 64 MiB it returns GP_ERR_INVALID_ARG and
 * launches nothing.  Metrics: MAE, MSE, RMSE, LOGLOSS, PEARSON (SPEARMAN:
 * GP_ERR_UNSUPPORTED).  Every call on a device shares that device's array
 * and overwrites it: calls that overlap on one device (other streams, other
 * threads' work in flight) race; a call ordered after another on the same
 * stream is safe.  The first call on a device looks up its array's address
 * (hipGetSymbolAddress) and its properties. */
gp_status gp_fitness_noalloc(const gp_population_dev* pop, const gp_dataset_dev* data,
                             gp_metric metric, float* fitness, void* stream);

/* Tournament selection (Sec. III-C1): tournament t draws tournament_size
 * program indices with replacement, draw d being floor(word * n / 2^32) for
 * word d%4 of Philox4x32-10(key = seed, counter = (d/4, t, generation, 0)),
 * and keeps the one with the best adjusted fitness
 *   raw + parsimony * len   (metric favouring smaller values), or
 *   raw - parsimony * len   (favouring larger values)  -- Eqs. (parsimony),
 * (fitness); float32 arithmetic with each operation rounded, the earliest draw
 * winning ties, NaN ranked worst.  fitness, len and winners are DEVICE
 * memory; winners[t] receives the winning program index. */
gp_status gp_tournament(const float* fitness, const int32_t* len, int32_t n_programs,
                        gp_metric metric, float parsimony, int32_t tournament_size,
                        int32_t n_tournaments, uint64_t seed, uint64_t generation,
                        int32_t* winners, void* stream);

/* Derivative of fitness with respect to every program constant (not in the
 * paper): grad_consts[const_off[p] + s] = g_p * d fitness_p / d consts[s],
 * with g_p = grad_fitness[p] (NULL: 1).  Reverse mode over each prefix list
 * per row, recomputing the forward values per row tile.  Local derivatives:
 * add (1,1), sub (1,-1), mul (b,a), div (1/b, -a/b^2) where |b| > 0.001 else 0,
 * log 1/a where |a| > 0.001 else 0, sqrt sign(a)/(2 sqrt|a|) (0 at a = 0),
 * sin cos a, cos -sin a, tan 1 + tan^2 a, neg -1; max / min (1,0) to the
 * selected operand (the first on ties or when the second is NaN), atan2
 * (b, -a)/(a^2+b^2) (0 at the origin), abs sign(a) (0 at 0), exp e^a, inv
 * -1/a^2 where |a| > 0.001 else 0, sq 2a, cube 3a^2, tanh 1 - tanh^2 a, atan
 * 1/(1+a^2), cbrt 1/(3 cbrt(a)^2) (0 at 0).  Metrics MAE, MSE, RMSE,
 * LOGLOSS, PEARSON.  fitness_out [n_programs] (nullable) receives the
 * fitness as gp_fitness would.  All pointers DEVICE memory.  The population
 * view must carry max_len (at most 2^25, else GP_ERR_INVALID_ARG) and
 * total_consts.  A program's constants in slots below 16 are summed in a
 * fixed order (bit-reproducible); further slots are summed with float64
 * atomics.  Rows per lane: a forced launch configuration's, else 2 or 4,
 * whichever keeps more rows in flight per CU at the kernel's occupancy.
 * Scratch grows with 2*max_len tape entries per wavefront (64 floats per
 * row per lane each). */
gp_status gp_fitness_backward(const gp_population_dev* pop, const gp_dataset_dev* data,
                              gp_metric metric, const float* grad_fitness,
                              float* fitness_out, float* grad_consts, void* stream);

/* ------------------------------------------------------------------ */
/* Genetic operations on the DEVICE.  The same draws, choices and      */
/* output layout as gp_plan_generation / gp_mutate (Sec. II-A, Sec.    */
/* III-C2; the paper mutates on the CPU): offspring agree with the     */
/* host functions bit for bit, with no host round trip.  Both calls    */
/* are asynchronous on `stream`, allocate nothing after their first    */
/* use at a size, and have fixed launch shapes (graph-capturable).     */
/* ------------------------------------------------------------------ */
/* An offspring population written by the device, in DEVICE memory. */
typedef struct {
    uint32_t* nodes;           /* [node_capacity]                                 */
    int64_t* prog_off;         /* [n_offspring + 1]                               */
    float* consts;             /* [const_capacity]                                */
    int64_t* const_off;        /* [n_offspring + 1]                               */
    int32_t* len;              /* [n_offspring]                                   */
    int64_t node_capacity;
    int64_t const_capacity;
} gp_population_out_dev;

/* gp_plan_generation with DEVICE outputs: ops and first_tournament
 * [n_offspring], n_tournaments [1]. */
gp_status gp_plan_generation_device(const gp_evolve_params* params, int32_t n_offspring,
                                    uint64_t generation, int32_t* ops, int32_t* first_tournament,
                                    int32_t* n_tournaments, void* stream);

/* gp_mutate on a DEVICE parent population (valid programs over
 * init->n_features, as gp_validate_population accepts; not re-checked) with
 * DEVICE ops, first_tournament [n_offspring] and winners [n_winners].  The
 * offspring go to `out`; info is DEVICE int64[4]: info[0], info[1] the total
 * nodes and constants; info[2] status bits -- 1: a capacity of `out` is
 * short, nothing was written; 2: an operation, tournament or winner index
 * was out of range, those offspring are the one-node program x0; 4: the
 * donors overflowed the library's bound (not reachable with settings that
 * pass the checks).  Subtree-mutation donors are bounded by 2^(max_depth+1)-1
 * nodes (tree methods) or max_len + 1 (exact length) each; settings whose
 * bound times n_offspring exceeds 2^25 nodes give GP_ERR_INVALID_ARG. */
gp_status gp_mutate_device(const gp_evolve_params* params, const gp_init_params* init,
                           const gp_population_dev* parents, const int32_t* ops,
                           const int32_t* first_tournament, const int32_t* winners, int32_t n_winners,
                           int32_t n_offspring, uint64_t generation, const gp_population_out_dev* out,
                           int64_t* info, void* stream);

/* ------------------------------------------------------------------ */
/* Launch configuration of the evaluation kernels (gp_evaluate,        */
/* gp_fitness).  A work item is one program on one chunk of rows; a    */
/* wavefront evaluates 64*rows_per_lane rows per pass ("tile").        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t rows_per_lane;    /* 1, 2 or 4                                         */
    int32_t feature_regs;     /* 0 (features read from memory), 2 or 8 (features
                                 held in registers; needs n_features <= it)        */
    int32_t tiles_per_chunk;  /* >= 1: rows per work item = 64*rows_per_lane*this  */
    int32_t waves_per_block;  /* 1, 2 or 4: block size 64, 128 or 256 threads     */
} gp_launch_config;

/* The configuration gp_fitness would use for this shape and metric on the
 * current device: the forced one if set, else the tuned one if the autotuner
 * has an entry for exactly (device, n_features, n_rows, n_programs, metric's
 * kernel), else the built-in heuristic. */
gp_status gp_get_launch_config(int32_t n_features, int64_t n_rows, int32_t n_programs,
                               gp_metric metric, gp_launch_config* out);

/* Force the configuration of every later gp_evaluate / gp_fitness call in this
 * process (all shapes); NULL returns to automatic selection.  Invalid values
 * give GP_ERR_INVALID_ARG; a feature_regs below a dataset's n_features makes
 * those calls fail with GP_ERR_INVALID_ARG. */
gp_status gp_set_launch_config(const gp_launch_config* cfg);

/* Limit on the device memory that Spearman fitness (Sec. III-C3: ranks from
 * a sort) uses for its batches of programs: 16 bytes per row per program
 * (sort keys and the values they carry, double-buffered; the program
 * outputs share the first key buffer), plus the sort's per-tile counts.  0 (the default) means 16 GiB and at most half the free
 * memory.  A batch holds at least one program whatever the limit.  Applies
 * to every later gp_fitness call and captured generation in this process;
 * results do not depend on it.  A negative value gives GP_ERR_INVALID_ARG. */
gp_status gp_set_spearman_workset(int64_t max_bytes);

/* Autotuner (batching of uneven programs; not in the paper).  Times the
 * fitness computation of this population under each candidate configuration
 * -- rows_per_lane 1, 2, 4; feature registers that fit n_features, and 0;
 * rows per work item from 1/4 to 2 times the heuristic's, at 4 waves per
 * block; then 1 and 2 waves per block for the best of those -- on the first
 * min(n_rows, 2^20) rows, `repeats` timed runs after one warm-up each, and
 * keeps the fastest for the full shape (device, n_features, n_rows,
 * n_programs, metric's kernel), which gp_fitness and gp_generation_run then
 * use unless a configuration is forced.  *best and *best_ms (nullable)
 * receive the choice and its time on the row prefix.  Synchronizes `stream`
 * and may allocate: not for use under stream capture.  Results are
 * unchanged by the choice except for the float64 summation order across row
 * chunks. */
gp_status gp_autotune(const gp_population_dev* pop, const gp_dataset_dev* data,
                      gp_metric metric, int32_t repeats, gp_launch_config* best,
                      double* best_ms, void* stream);

/* The tuned entries as JSON lines (one object per shape, keys arch, n_cu,
 * n_features, n_rows, n_programs, kernel, rows_per_lane, feature_regs,
 * tiles_per_chunk, waves_per_block, ms); load merges a file written by save (a malformed line
 * gives GP_ERR_INVALID_ARG and loads nothing); clear forgets every entry. */
gp_status gp_autotune_save(const char* path);
gp_status gp_autotune_load(const char* path);
gp_status gp_autotune_clear(void);

/* ------------------------------------------------------------------ */
/* One generation as a HIP graph (batching; the paper's future-work    */
/* item of fewer transfers, Sec. V).  The graph holds: one upload of   */
/* the whole population from pinned host memory (instead of copies per */
/* program, Sec. III-D2), the fitness computation of gp_fitness, the   */
/* tournaments of gp_tournament (Sec. III-C1) and the download of      */
/* fitness and winners.  It is captured on the first run, after the    */
/* autotuner if asked, at the capacities given here, and replayed for  */
/* every later generation; the generation number the tournaments use   */
/* travels with the population.                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n_programs;        /* population size, fixed across generations (>= 1) */
    int64_t node_capacity;     /* bound on sum(len) of any generation              */
    int64_t const_capacity;    /* bound on the constants of any generation         */
    int32_t metric;            /* gp_metric (SPEARMAN: no autotune, no kernel time) */
    float parsimony;
    int32_t tournament_size;   /* >= 1                                              */
    int32_t n_tournaments;     /* winners per generation (>= 0)                     */
    uint64_t seed;             /* Philox key of the tournaments                     */
    int32_t autotune;          /* 1: tune on the first population (unless forced)  */
    int32_t time_kernel;       /* 1: time the evaluation kernel inside the graph
                                  (device wall clock read just before and after it) */
} gp_generation_params;

typedef struct gp_generation_s gp_generation;

/* Allocates the pinned staging and result buffers (about node_capacity*4 +
 * const_capacity*4 + 20*n_programs bytes on host and device), a stream of
 * its own and a private scratch arena.  The dataset (DEVICE memory) must
 * outlive the object. */
gp_status gp_generation_create(const gp_generation_params* params, const gp_dataset_dev* data,
                               gp_generation** out);

/* Runs one generation on the HOST population given (same flat layout as
 * gp_build_population, n_programs programs): validates it
 * (gp_validate_population; GP_ERR_BUFFER_TOO_SMALL beyond the capacities),
 * stages it, launches the graph, waits, and copies fitness[n_programs] and
 * winners[n_tournaments] (HOST, nullable) out.  Winners equal those of
 * gp_tournament(seed, generation) on the same fitness.  Calls on one object
 * must not overlap; the device current at creation must be current. */
gp_status gp_generation_run(gp_generation* gen, const uint32_t* nodes, const int64_t* prog_off,
                            const float* consts, const int64_t* const_off, const int32_t* len,
                            uint64_t generation, float* fitness, int32_t* winners);

/* The launch configuration captured; the evaluation kernel's duration in the
 * last run (ms, -1 unless time_kernel) measured by HIP event-record nodes
 * placed around it in the graph (*timed_by_events = 1), or by the device
 * clock if HIP refused those nodes (*timed_by_events = 0); the clock-stamp
 * duration itself; and the autotuner's best time (ms on the row prefix, -1
 * if not tuned).  Each output is nullable. */
gp_status gp_generation_info(const gp_generation* gen, gp_launch_config* cfg, float* kernel_ms,
                             float* clock_ms, int32_t* timed_by_events, double* tuned_ms);

/* Waits for the object's work and frees it (NULL is ignored). */
void gp_generation_destroy(gp_generation* gen);

/* ------------------------------------------------------------------ */
/* A device-resident generational loop (Alg. 1 with the Sec. III-C     */
/* order; the paper mutates on the CPU, here nothing leaves the        */
/* device).  Two populations alternate as parents and offspring.  Each */
/* generation is one replay of a captured graph: fitness of the        */
/* current population (gp_fitness), the fitness recorded in a device   */
/* history, 2 * n_programs tournaments (gp_tournament; a generation    */
/* uses the first ones it needs, which are the same as if only those   */
/* had run), the operation pre-draw (gp_plan_generation_device) and    */
/* the genetic operations (gp_mutate_device).  The generation number   */
/* lives in device memory.  At the same launch configuration every     */
/* generation equals gp_fitness + gp_tournament + gp_plan_generation + */
/* gp_mutate on the host, bit for bit.                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n_programs;        /* population size (1 .. 2^29)                        */
    int32_t metric;            /* gp_metric (SPEARMAN: no autotune, no kernel time)   */
    float parsimony;
    int32_t tournament_size;   /* >= 1                                                */
    uint64_t tournament_seed;  /* Philox key of the tournaments                       */
    gp_evolve_params evolve;
    gp_init_params init;       /* donors of subtree mutation, point-mutation sets;   */
                               /* init.n_features must equal the dataset's           */
    int32_t max_generations;   /* history capacity: max_generations + 1 entries        */
    int32_t autotune;          /* 1: tune on the initial population (unless forced)  */
    int32_t time_kernel;       /* 1: HIP event nodes around the evaluation kernel     */
    uint64_t first_generation; /* generation number of the initial population: a run
                                  resumed from generation g's population passes g and
                                  continues exactly (the draws are counter-based)     */
} gp_evolution_params;

typedef struct gp_evolution_s gp_evolution;

/* Uploads the HOST initial population (validated; every program at most
 * max(evolve.max_len, its longest program) nodes is what the offspring
 * buffers hold: each population is allocated at n_programs times that).
 * The dataset (DEVICE memory) must outlive the object. */
gp_status gp_evolution_create(const gp_evolution_params* params, const gp_dataset_dev* data,
                              const uint32_t* nodes, const int64_t* prog_off, const float* consts,
                              const int64_t* const_off, const int32_t* len, gp_evolution** out);

/* Runs generations g .. g + n - 1 (g = first_generation + the generations run
 * so far): for each, the current population's fitness is recorded as history
 * entry g - first_generation and its offspring become the current
 * population.  Waits for the device;
 * GP_ERR_DEVICE if a mutation status bit was raised (see gp_mutate_device),
 * GP_ERR_INVALID_ARG beyond max_generations. */
gp_status gp_evolution_run(gp_evolution* evo, int32_t n_generations);

/* Fitness of the current population, recorded as its history entry, without
 * selection or mutation (the loop's last step).  Waits for the device. */
gp_status gp_evolution_evaluate(gp_evolution* evo);

/* The history: *n_recorded entries; fitness_history [n_recorded *
 * n_programs] (generation first_generation + k in row k) and nodes_history
 * [n_recorded] (the sum of lengths of that generation), HOST, nullable, at
 * most `capacity` entries copied. */
gp_status gp_evolution_history(const gp_evolution* evo, int32_t capacity, int32_t* n_recorded,
                               float* fitness_history, int64_t* nodes_history);

/* The current population to HOST buffers (the gp_mutate layout);
 * GP_ERR_BUFFER_TOO_SMALL with the totals set if a capacity is short. */
gp_status gp_evolution_population(const gp_evolution* evo, uint32_t* nodes, int64_t nodes_cap,
                                  int64_t* prog_off, float* consts, int64_t consts_cap,
                                  int64_t* const_off, int32_t* len, int64_t* total_nodes,
                                  int64_t* total_consts);

/* Launch configuration, the evaluation kernel's duration in the last
 * replay (ms, -1 unless time_kernel and the event nodes were accepted),
 * the generations run by this object, and the autotuner's best time (-1 if
 * not tuned).
 * Each output is nullable. */
gp_status gp_evolution_info(const gp_evolution* evo, gp_launch_config* cfg, float* kernel_ms,
                            int64_t* generation, double* tuned_ms);

/* Waits for the object's work and frees it (NULL is ignored). */
void gp_evolution_destroy(gp_evolution* evo);

/* ------------------------------------------------------------------ */
/* Kernel timing.  While enabled, the library brackets every launch of */
/* its evaluation kernel (the dominant kernel of gp_evaluate and       */
/* gp_fitness) with HIP events on the caller's stream.                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t launches;         /* evaluation-kernel launches since enabled   */
    double total_ms;          /* their summed event-measured duration (ms)  */
    int64_t node_rows;        /* sum over launches of sum(len) * n_rows     */
} gp_profile;

/* enable != 0 starts (and resets) the record; 0 stops it. */
gp_status gp_profile_enable(int enable);
/* Waits for the recorded events, then fills *out. */
gp_status gp_profile_read(gp_profile* out);

#ifdef __cplusplus
}
#endif
#endif /* GP_H */
