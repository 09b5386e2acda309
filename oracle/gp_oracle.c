/*
 * gp_oracle.c -- plain, slow, obviously-correct CPU oracle for stack-based
 * genetic-programming evaluation ("Accelerating Genetic Programming using
 * GPUs", arXiv 2110.11226).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no header, helper, table or
 * generator with the GPU library: every constant below is written out here
 * from the paper (or from the reading of it that the design notes record).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no FTZ/DAZ, no contraction: every float operation is a single IEEE op).
 *
 * What it computes (each function cites the passage it follows):
 *   - program value of a prefix list on one row, by the right-to-left stack
 *     scan of Sec. III-A, in float32 and in float64, over 21 functions (the
 *     paper's experiments use +, -, *, protected /, sin, cos, tan; Sec. III-D1
 *     counts 33 without listing them; the others here follow gplearn, the
 *     library the paper compares against);
 *   - per-program fitness under the weighted metrics of Sec. III-C3
 *     (MAE, MSE, RMSE, logistic loss, Pearson, Spearman);
 *   - tournament selection with the parsimony penalty, Sec. III-C1,
 *     Eqs. (parsimony) and (fitness);
 *   - Philox4x32-10 (the counter-based generator cited in Sec. III-B);
 *   - the Full / Grow / ramped-half-and-half initialisations of Sec. II-A and
 *     an exact-length generator (not in the paper);
 *   - float64 reverse-mode derivatives of fitness with respect to program
 *     constants (not in the paper).
 *
 * Parity status: every function here is pinned by tests/test_oracle_*.py
 * against closed forms, hand-evaluated programs, brute force or an
 * independent library routine, except where a comment says "parity unpinned".
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- node encoding (reading: op in bits 0-7, argument in bits 8-31) ---- */
enum {
    O_VAR = 0, O_CONST = 1,
    O_ADD = 2, O_SUB = 3, O_MUL = 4, O_DIV = 5,
    O_NEG = 6, O_LOG = 7, O_SQRT = 8, O_SIN = 9, O_COS = 10, O_TAN = 11,
    O_MAX = 12, O_MIN = 13, O_ATAN2 = 14,
    O_ABS = 15, O_EXP = 16, O_INV = 17, O_SQ = 18, O_CUBE = 19, O_TANH = 20, O_ATAN = 21, O_CBRT = 22,
    O_NUM = 23,
    /* user-defined functions (Sec. V, custom function sets): 24..27 take one
     * argument, 28..31 two; each is defined by orc_set_user_function */
    O_USER1 = 24, O_USER2 = 28, O_LIMIT = 32
};
#define ORC_STACK 20          /* fixed evaluation stack, Sec. III-B */

static int op_arity(int op)
{
    switch (op) {
    case O_VAR: case O_CONST: return 0;
    case O_ADD: case O_SUB: case O_MUL: case O_DIV: case O_MAX: case O_MIN: case O_ATAN2: return 2;
    case O_NEG: case O_LOG: case O_SQRT: case O_SIN: case O_COS: case O_TAN:
    case O_ABS: case O_EXP: case O_INV: case O_SQ: case O_CUBE: case O_TANH: case O_ATAN: case O_CBRT:
        return 1;
    default:
        if (op >= O_USER1 && op < O_USER2) return 1;
        if (op >= O_USER2 && op < O_LIMIT) return 2;
        return -1;
    }
}

/* ---- user-defined functions (Sec. V: custom function sets and losses) ----
 * Function u (opcode O_USER1 + u) is a prefix list over the built-in
 * functions in which VAR k stands for its argument k and CONST k for its
 * constant k.  Its value on arguments (a, b) is the value of that list with
 * the arguments put in: evaluated here by the same right-to-left stack
 * rule as a program, every built-in operation rounded to float32 (float32
 * path) or carried in float64.  Definitions are not checked here (the
 * library's gp_register_function checks them). */
#define ORC_USER_NODES 32
#define ORC_USER_CONSTS 16
static struct {
    int len;
    uint32_t nodes[ORC_USER_NODES];
    float consts[ORC_USER_CONSTS];
} orc_user[O_LIMIT - O_USER1];

int orc_set_user_function(int op, const uint32_t *nodes, int len, const float *consts, int n_consts)
{
    if (op < O_USER1 || op >= O_LIMIT || len < 0 || len > ORC_USER_NODES || n_consts < 0 ||
        n_consts > ORC_USER_CONSTS)
        return -1;
    int u = op - O_USER1;
    orc_user[u].len = len;
    for (int i = 0; i < ORC_USER_NODES; ++i) orc_user[u].nodes[i] = i < len ? nodes[i] : 0u;
    for (int i = 0; i < ORC_USER_CONSTS; ++i) orc_user[u].consts[i] = i < n_consts ? consts[i] : 0.0f;
    return 0;
}

static float op_f32(int op, float a, float b);
static double op_f64(int op, double a, double b);

static float user_f32(int op, float a, float b)
{
    int u = op - O_USER1;
    float st[ORC_USER_NODES];
    int h = 0;
    for (int i = orc_user[u].len - 1; i >= 0; --i) {
        int dop = (int)(orc_user[u].nodes[i] & 0xffu);
        uint32_t arg = orc_user[u].nodes[i] >> 8;
        if (dop == O_VAR) { st[h++] = arg == 0 ? a : b; continue; }
        if (dop == O_CONST) { st[h++] = orc_user[u].consts[arg % ORC_USER_CONSTS]; continue; }
        int ar = op_arity(dop);
        if (ar < 1 || dop >= O_NUM || h < ar) return NAN;
        float x = st[--h];
        float y = ar == 2 ? st[--h] : 0.0f;
        st[h++] = op_f32(dop, x, y);
    }
    return h == 1 ? st[0] : NAN;
}

static double user_f64(int op, double a, double b)
{
    int u = op - O_USER1;
    double st[ORC_USER_NODES];
    int h = 0;
    for (int i = orc_user[u].len - 1; i >= 0; --i) {
        int dop = (int)(orc_user[u].nodes[i] & 0xffu);
        uint32_t arg = orc_user[u].nodes[i] >> 8;
        if (dop == O_VAR) { st[h++] = arg == 0 ? a : b; continue; }
        if (dop == O_CONST) { st[h++] = (double)orc_user[u].consts[arg % ORC_USER_CONSTS]; continue; }
        int ar = op_arity(dop);
        if (ar < 1 || dop >= O_NUM || h < ar) return NAN;
        double x = st[--h];
        double y = ar == 2 ? st[--h] : 0.0;
        st[h++] = op_f64(dop, x, y);
    }
    return h == 1 ? st[0] : NAN;
}

/* ---- protected operators (reading: the gplearn convention) ---- */
static const float ORC_EPS = 0.001f;      /* float nearest 0.001 */

static float cr_f32(int op, float a, float b);
static float pdiv_f(float a, float b) { return fabsf(b) > ORC_EPS ? a / b : 1.0f; }
static float plog_f(float a) { return fabsf(a) > ORC_EPS ? cr_f32(O_LOG, fabsf(a), 0.0f) : 0.0f; }
static float psqrt_f(float a) { return sqrtf(fabsf(a)); }

static double pdiv_d(double a, double b) { return fabs(b) > (double)ORC_EPS ? a / b : 1.0; }
static double plog_d(double a) { return fabs(a) > (double)ORC_EPS ? log(fabs(a)) : 0.0; }
static double psqrt_d(double a) { return sqrt(fabs(a)); }

/* ---- the wider function set (reading: the paper counts its functions,
 * Sec. III-D1, without listing them).  max / min follow IEEE maxNum /
 * minNum (fmax / fmin: a NaN operand yields the other); atan2 takes the
 * first operand as y; inv is protected like division (0 where |a| <=
 * 0.001, gplearn's convention); sq is a*a and cube (a*a)*a, rounded after
 * each product; exp, tanh, atan, cbrt are the library functions. ---- */
static float pinv_f(float a) { return fabsf(a) > ORC_EPS ? 1.0f / a : 0.0f; }
static double pinv_d(double a) { return fabs(a) > (double)ORC_EPS ? 1.0 / a : 0.0; }

/* result of function `op` on its first operand a and (binary) second b */
/* max / min as IEEE 754-2019 maximumNumber / minimumNumber: a NaN operand
 * is ignored and -0 orders below +0 (C's fmax leaves the sign of a zero
 * result open, and atan2 can see it) */
static float max_f(float a, float b)
{
    if (isnan(a)) return b;
    if (isnan(b)) return a;
    if (a > b) return a;
    if (b > a) return b;
    return signbit(a) ? b : a;
}
static float min_f(float a, float b)
{
    if (isnan(a)) return b;
    if (isnan(b)) return a;
    if (a < b) return a;
    if (b < a) return b;
    return signbit(a) ? a : b;
}
static double max_d(double a, double b)
{
    if (isnan(a)) return b;
    if (isnan(b)) return a;
    if (a > b) return a;
    if (b > a) return b;
    return signbit(a) ? b : a;
}
static double min_d(double a, double b)
{
    if (isnan(a)) return b;
    if (isnan(b)) return a;
    if (a < b) return a;
    if (b < a) return b;
    return signbit(a) ? a : b;
}

/* ---- correctly rounded float32 values of the library functions ----
 * Reading (float32 semantics): the float32 evaluation rounds the exact value
 * of every function once, to nearest (ties to even), as IEEE arithmetic does
 * for +, -, *, / and sqrt.  The paper names its functions but no library,
 * and the float32 value of a program would otherwise depend on which
 * library computed sin.  The C library's double result (within a few of its
 * ulps of the exact value) decides the rounding unless it lies within
 * 8 of its ulps (orc_cr_set_margin) of a float32 rounding boundary; then the x87
 * extended-precision result decides, and if that too lies that close to the
 * boundary the case is counted in orc_cr_undecided() (the extended result's
 * rounding is returned). */
static double g_cr_margin = 8.0;   /* tests widen it to exercise the fallback */
static long long g_cr_undecided = 0;

long long orc_cr_undecided(void) { return g_cr_undecided; }
void orc_cr_reset(void) { g_cr_undecided = 0; }
void orc_cr_set_margin(double m) { g_cr_margin = m > 0.0 ? m : 8.0; }

/* the float32 rounding boundaries on either side of f = RN(v), as doubles
 * (exact: a midpoint of two floats has 25 significant bits); the boundary
 * beyond FLT_MAX is FLT_MAX + half its spacing */
static void f32_boundaries(float f, double *lo, double *hi)
{
    const double top = 0x1.ffffffp127;
    if (isinf(f)) {
        *lo = f > 0 ? top : -INFINITY;
        *hi = f > 0 ? INFINITY : -top;
        return;
    }
    float fd = nextafterf(f, -INFINITY), fu = nextafterf(f, INFINITY);
    *lo = isinf(fd) ? -top : ((double)f + (double)fd) * 0.5;
    *hi = isinf(fu) ? top : ((double)f + (double)fu) * 0.5;
}

static int near_boundary_d(double v)
{
    if (isnan(v)) return 0;
    double lo, hi;
    f32_boundaries((float)v, &lo, &hi);
    double d = fmin(v - lo, hi - v);
    double a = fabs(v);
    double ulp = isinf(a) ? 0.0 : nextafter(a, INFINITY) - a;
    return d <= g_cr_margin * ulp;
}

static int near_boundary_ld(long double v)
{
    if (isnan(v)) return 0;
    double lo, hi;
    f32_boundaries((float)v, &lo, &hi);
    long double d = fminl(v - (long double)lo, (long double)hi - v);
    long double a = fabsl(v);
    long double ulp = isinf(a) ? 0.0L : nextafterl(a, INFINITY) - a;
    return d <= 8.0L * ulp;
}

static double lib_d(int op, double a, double b)
{
    switch (op) {
    case O_SIN: return sin(a);
    case O_COS: return cos(a);
    case O_TAN: return tan(a);
    case O_LOG: return log(a);
    case O_EXP: return exp(a);
    case O_TANH: return tanh(a);
    case O_ATAN: return atan(a);
    case O_CBRT: return cbrt(a);
    case O_ATAN2: return atan2(a, b);
    default: return NAN;
    }
}

static long double lib_ld(int op, long double a, long double b)
{
    switch (op) {
    case O_SIN: return sinl(a);
    case O_COS: return cosl(a);
    case O_TAN: return tanl(a);
    case O_LOG: return logl(a);
    case O_EXP: return expl(a);
    case O_TANH: return tanhl(a);
    case O_ATAN: return atanl(a);
    case O_CBRT: return cbrtl(a);
    case O_ATAN2: return atan2l(a, b);
    default: return NAN;
    }
}

/* RN(f(a[, b])) for the library function op */
static float cr_f32(int op, float a, float b)
{
    double v = lib_d(op, (double)a, (double)b);
    if (!near_boundary_d(v)) return (float)v;
    long double w = lib_ld(op, (long double)a, (long double)b);
    if (near_boundary_ld(w)) {
#pragma omp atomic
        g_cr_undecided++;
    }
    return (float)w;
}

static float op_f32(int op, float a, float b)
{
    switch (op) {
    case O_ADD: return a + b;
    case O_SUB: return a - b;
    case O_MUL: return a * b;
    case O_DIV: return pdiv_f(a, b);
    case O_MAX: return max_f(a, b);
    case O_MIN: return min_f(a, b);
    case O_ATAN2: return cr_f32(O_ATAN2, a, b);
    case O_NEG: return -a;
    case O_LOG: return plog_f(a);
    case O_SQRT: return psqrt_f(a);
    case O_SIN: case O_COS: case O_TAN: case O_EXP: case O_TANH: case O_ATAN: case O_CBRT:
        return cr_f32(op, a, 0.0f);
    case O_ABS: return fabsf(a);
    case O_INV: return pinv_f(a);
    case O_SQ: return a * a;
    case O_CUBE: { float q = a * a; return q * a; }
    default: return (op >= O_USER1 && op < O_LIMIT) ? user_f32(op, a, b) : NAN;
    }
}

static double op_f64(int op, double a, double b)
{
    switch (op) {
    case O_ADD: return a + b;
    case O_SUB: return a - b;
    case O_MUL: return a * b;
    case O_DIV: return pdiv_d(a, b);
    case O_MAX: return max_d(a, b);
    case O_MIN: return min_d(a, b);
    case O_ATAN2: return atan2(a, b);
    case O_NEG: return -a;
    case O_LOG: return plog_d(a);
    case O_SQRT: return psqrt_d(a);
    case O_SIN: return sin(a);
    case O_COS: return cos(a);
    case O_TAN: return tan(a);
    case O_ABS: return fabs(a);
    case O_EXP: return exp(a);
    case O_INV: return pinv_d(a);
    case O_SQ: return a * a;
    case O_CUBE: return a * a * a;
    case O_TANH: return tanh(a);
    case O_ATAN: return atan(a);
    case O_CBRT: return cbrt(a);
    default: return (op >= O_USER1 && op < O_LIMIT) ? user_f64(op, a, b) : NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Validation: right-to-left stack-height scan (Sec. III-A: the list is read  */
/* in reverse; Sec. III-C2: a stack of size m bounds what can be evaluated).  */
/* Returns 0 if valid; 1 bad opcode; 2 stack underflow / not exactly one      */
/* result; 3 stack height above ORC_STACK; 4 feature index out of range;      */
/* 5 constant slot out of range; 6 empty program.                             */
/* ------------------------------------------------------------------------ */
int orc_check_program(const uint32_t *nodes, int64_t len, int32_t n_features,
                      int64_t n_consts, int32_t *max_height)
{
    int64_t h = 0, hmax = 0;
    if (len <= 0) return 6;
    for (int64_t i = len - 1; i >= 0; --i) {
        int op = (int)(nodes[i] & 0xffu);
        uint32_t arg = nodes[i] >> 8;
        int a = op_arity(op);
        if (a < 0) return 1;
        if (op == O_VAR && (int64_t)arg >= n_features) return 4;
        if (op == O_CONST && (int64_t)arg >= n_consts) return 5;
        if (h < a) return 2;
        h = h - a + 1;
        if (h > hmax) hmax = h;
        if (h > ORC_STACK) return 3;
    }
    if (h != 1) return 2;
    if (max_height) *max_height = (int32_t)hmax;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Evaluation of one program on one row (Sec. III-A, III-C3 execution step):  */
/* scan the prefix list from its last node to its first; a terminal pushes   */
/* its value; a function pops its operands -- the first pop is its first      */
/* argument, because in prefix order the first child is written first and so */
/* is evaluated last -- and pushes its result.  The one value left is the     */
/* program's output.                                                          */
/* ------------------------------------------------------------------------ */
static float eval_row_f32(const uint32_t *nodes, int64_t len, const float *c,
                          const float *X, int64_t ld, int64_t row)
{
    float st[ORC_STACK];
    int h = 0;
    for (int64_t i = len - 1; i >= 0; --i) {
        int op = (int)(nodes[i] & 0xffu);
        uint32_t arg = nodes[i] >> 8;
        int ar = op_arity(op);
        if (op == O_VAR) { st[h++] = X[(int64_t)arg * ld + row]; continue; }
        if (op == O_CONST) { st[h++] = c[arg]; continue; }
        if (ar < 0) return NAN;
        float a = st[--h];
        float b = ar == 2 ? st[--h] : 0.0f;
        st[h++] = op_f32(op, a, b);
    }
    return st[0];
}

static double eval_row_f64(const uint32_t *nodes, int64_t len, const float *c,
                           const float *X, int64_t ld, int64_t row)
{
    double st[ORC_STACK];
    int h = 0;
    for (int64_t i = len - 1; i >= 0; --i) {
        int op = (int)(nodes[i] & 0xffu);
        uint32_t arg = nodes[i] >> 8;
        int ar = op_arity(op);
        if (op == O_VAR) { st[h++] = (double)X[(int64_t)arg * ld + row]; continue; }
        if (op == O_CONST) { st[h++] = (double)c[arg]; continue; }
        if (ar < 0) return NAN;
        double a = st[--h];
        double b = ar == 2 ? st[--h] : 0.0;
        st[h++] = op_f64(op, a, b);
    }
    return st[0];
}

/* Conditioning analysis of one row (test infrastructure for the tolerance
 * policy).  Evaluates the program in float32 and float64 in lock-step and
 * carries, in float64, a bound E on how far another float32 evaluation can
 * move when every library-function result (sin, cos, tan, log, exp, tanh,
 * atan, cbrt, atan2) that it does not round correctly is allowed to differ
 * from the correctly rounded one by `u` relative (an implementation within a
 * few ulp); the functions in exact_mask (bit per opcode, argument xm), and
 * add, sub, mul, div, neg, abs, sqrt, max, min, inv, sq and cube, are
 * correctly rounded on both sides and contribute nothing of their own.  Operands carry bounds Ea, Eb; each node's bound is the largest
 * change of its value over the whole box [a - Ea, a + Ea] x [b - Eb, b + Eb]
 * (mean value theorem with the supremum of |f'| over the interval, or the
 * exact remainder of a polynomial), not the first-order |f'(a)| Ea, so that
 * it stays a bound where a large Ea meets a saturating function:
 *   terminal 0;  a+b, a-b: Ea+Eb;  a*b: |b|Ea + |a|Eb + Ea Eb;
 *   a/b: (Ea|b| + |a|Eb) / (|b|(|b|-Eb)) (0 on the protected arm);
 *   -a, |a|: Ea;  max, min: max(Ea, Eb) (1-Lipschitz in each operand);
 *   sqrt|a|: min(Ea / (2 sqrt(|a|-Ea)), sqrt(Ea));  inv: Ea/(|a|-Ea)^2;
 *   a^2: 2|a|Ea + Ea^2;  a^3: 3a^2 Ea + 3|a|Ea^2 + Ea^3;
 *   f(a) for the library functions: D (1+u) + u |f(a)| with D = Ea sup|f'|
 *   (cbrt also min'd with its Hoelder bound 2^(2/3) Ea^(1/3));
 *   atan2(a, b): D = ((|b|+Eb) Ea + (|a|+Ea) Eb) / rmin^2, rmin the distance
 *   of the box from the origin, and a possible jump of 2 pi (near) when
 *   b < 0 and a lies within Ea of 0.
 * A bound that cannot be given (the interval reaches a pole or the origin)
 * is infinite, which excludes the row.
 * Outputs: *v32, *v64 the two values, *E the bound on the output, *flip if
 * a protected predicate or a sign that selects a branch of atan2 came out
 * differently in float32 and float64, *near if a protected predicate's
 * operand lies within its own bound of the 0.001 threshold, or a value
 * within its bound of float32 overflow (so two float32 evaluations may take
 * different arms). */
static double mul0(double x, double y) { return (x == 0.0 || y == 0.0) ? 0.0 : x * y; }

static const double ORC_PI = 3.14159265358979323846;

/* does [lo, hi] contain off + k pi for some integer k? */
static int has_point(double lo, double hi, double off)
{
    if (!(hi - lo < ORC_PI)) return 1;
    double k = ceil((lo - off) / ORC_PI);
    return off + k * ORC_PI <= hi;
}

/* sup |f'(t)| over t in [a - e, a + e], e > 0, for the library functions */
static double sup_deriv(int op, double a, double e)
{
    double lo = a - e, hi = a + e, m = fabs(a) - e;
    double nearest = (lo <= 0.0 && hi >= 0.0) ? 0.0 : fmin(fabs(lo), fabs(hi));
    switch (op) {
    case O_SIN: return has_point(lo, hi, 0.0) ? 1.0 : fmax(fabs(cos(lo)), fabs(cos(hi)));
    case O_COS: return has_point(lo, hi, ORC_PI / 2) ? 1.0 : fmax(fabs(sin(lo)), fabs(sin(hi)));
    case O_TAN: {
        if (has_point(lo, hi, ORC_PI / 2)) return INFINITY;
        double tl = tan(lo), th = tan(hi);
        return fmax(1.0 + tl * tl, 1.0 + th * th);
    }
    case O_LOG: return m > 0.0 ? 1.0 / m : INFINITY;
    case O_EXP: return exp(hi);
    case O_TANH: { double t = tanh(nearest); return 1.0 - t * t; }
    case O_ATAN: return 1.0 / (1.0 + nearest * nearest);
    case O_CBRT: return m > 0.0 ? 1.0 / (3.0 * cbrt(m) * cbrt(m)) : INFINITY;
    default: return INFINITY;
    }
}

/* A correctly rounded operation whose operands differ between the two
 * sides (bound e > 0) may also round them to neighbouring floats: one
 * spacing of the result, at most rf (|v| + e) with rf = 2^-23 for float32,
 * per rounding.  Operands known exactly on both sides round identically. */
static double round_flip(double v, double e, int n_round, double rf)
{
    return e > 0.0 ? n_round * rf * (fabs(v) + e) : 0.0;
}

/* the sign bit as 0 / 1 (signbit() returns an unspecified nonzero value,
 * which may differ between a float and a double argument) */
static int neg_bit(double x) { return signbit(x) ? 1 : 0; }

/* bound of a library function's result: D (1 + u) + u |v| */
static double lib_bound(double D, double v, double u) { return D * (1.0 + u) + u * fabs(v); }

/* bound of a library function's result when both sides round it correctly
 * (bit `op` of exact_mask): only the operand's movement D and, where the
 * operand moves, a flip to the neighbouring float */
static double fn_bound(int op, uint32_t exact_mask, double D, double v, double u, double rf)
{
    if (exact_mask & (1u << op)) return D + round_flip(v, D, 1, rf);
    return lib_bound(D, v, u);
}

static void row_analysis(const uint32_t *nodes, int64_t len, const float *c,
                         const float *X, int64_t ld, int64_t row, double u, double rf, uint32_t xm,
                         float *v32, double *v64, double *Eout, int *flip_out, int *near_out)
{
    float sf[ORC_STACK];
    double sd[ORC_STACK], se[ORC_STACK];
    int h = 0, flip = 0, near = 0;
    const double eps = (double)ORC_EPS;
    for (int64_t i = len - 1; i >= 0; --i) {
        int op = (int)(nodes[i] & 0xffu);
        uint32_t arg = nodes[i] >> 8;
        float af, bf;
        double ad, bd, ea, eb;
        switch (op) {
        case O_VAR:
            sf[h] = X[(int64_t)arg * ld + row]; sd[h] = (double)sf[h]; se[h] = 0.0; h++; break;
        case O_CONST:
            sf[h] = c[arg]; sd[h] = (double)c[arg]; se[h] = 0.0; h++; break;
        case O_ADD: case O_SUB: case O_MUL: case O_DIV: case O_MAX: case O_MIN: case O_ATAN2:
            h--; af = sf[h]; ad = sd[h]; ea = se[h];
            h--; bf = sf[h]; bd = sd[h]; eb = se[h];
            sf[h] = op_f32(op, af, bf); sd[h] = op_f64(op, ad, bd);
            if (op == O_MAX || op == O_MIN) {
                se[h] = ea > eb ? ea : eb;
            } else if (op == O_ATAN2) {
                /* the branch cut on the negative x axis: a sign of the first
                 * operand that differs between the two paths, or lies within
                 * its bound of zero, moves the result by about 2 pi */
                if ((neg_bit(bf) || neg_bit(bd)) && neg_bit(af) != neg_bit(ad)) flip = 1;
                if (af == 0.0f && ad == 0.0 && neg_bit(bf) != neg_bit(bd)) flip = 1;
                if (bd < 0.0 && fabs(ad) <= ea) near = 1;
                if (ea == 0.0 && eb == 0.0) {
                    se[h] = fn_bound(O_ATAN2, xm, 0.0, sd[h], u, rf);
                } else {
                    double ra = fmax(fabs(ad) - ea, 0.0), rb = fmax(fabs(bd) - eb, 0.0);
                    double r2 = ra * ra + rb * rb;
                    if (!(r2 > 0.0)) { near = 1; se[h] = INFINITY; }
                    else se[h] = fn_bound(O_ATAN2, xm, (mul0(fabs(bd) + eb, ea) + mul0(fabs(ad) + ea, eb)) / r2,
                                          sd[h], u, rf);
                }
            } else if (op == O_ADD || op == O_SUB) {
                se[h] = ea + eb;
                se[h] += round_flip(sd[h], se[h], 1, rf);
            } else if (op == O_MUL) {
                se[h] = mul0(fabs(bd), ea) + mul0(fabs(ad), eb) + mul0(ea, eb);
                se[h] += round_flip(sd[h], se[h], 1, rf);
            } else {
                if ((fabsf(bf) > ORC_EPS) != (fabs(bd) > eps)) flip = 1;
                if (eb > 0.0 && fabs(fabs((double)bf) - eps) <= eb) near = 1;
                if (!(fabs(bd) > eps)) se[h] = 0.0;
                else if (eb >= fabs(bd)) se[h] = INFINITY;
                else se[h] = (mul0(ea, fabs(bd)) + mul0(fabs(ad), eb)) / (fabs(bd) * (fabs(bd) - eb));
                se[h] += round_flip(sd[h], se[h], 1, rf);
            }
            h++;
            break;
        default:
            h--; af = sf[h]; ad = sd[h]; ea = se[h];
            if (op < 0 || op >= O_NUM || op_arity(op) != 1) {
                *v32 = NAN; *v64 = NAN; *Eout = INFINITY; *flip_out = 1; *near_out = 1; return;
            }
            sf[h] = op_f32(op, af, 0.0f); sd[h] = op_f64(op, ad, 0.0);
            switch (op) {
            case O_NEG: case O_ABS: se[h] = ea; break;
            case O_LOG: case O_INV:
                if ((fabsf(af) > ORC_EPS) != (fabs(ad) > eps)) flip = 1;
                if (ea > 0.0 && fabs(fabs((double)af) - eps) <= ea) near = 1;
                if (!(fabs(ad) > eps)) se[h] = 0.0;            /* the protected arm: a constant */
                else if (op == O_INV) {
                    double m = fabs(ad) - ea;
                    se[h] = ea == 0.0 ? 0.0 : (m > 0.0 ? ea / (m * m) : INFINITY);
                    se[h] += round_flip(sd[h], se[h], 1, rf);
                } else {
                    se[h] = fn_bound(O_LOG, xm, ea == 0.0 ? 0.0 : ea * sup_deriv(O_LOG, ad, ea), sd[h], u, rf);
                }
                break;
            case O_SQRT: {
                double m = fabs(ad) - ea;
                se[h] = ea == 0.0 ? 0.0 : fmin(m > 0.0 ? ea / (2.0 * sqrt(m)) : INFINITY, sqrt(ea));
                se[h] += round_flip(sd[h], se[h], 1, rf);
                break;
            }
            case O_SQ:
                se[h] = mul0(2.0 * fabs(ad), ea) + mul0(ea, ea);
                se[h] += round_flip(sd[h], se[h], 1, rf);
                break;
            case O_CUBE:   /* two roundings: (a*a)*a */
                se[h] = mul0(3.0 * ad * ad, ea) + mul0(3.0 * fabs(ad), mul0(ea, ea)) + mul0(ea, mul0(ea, ea));
                se[h] += round_flip(sd[h], se[h], 2, rf);
                break;
            case O_CBRT: {
                double D = ea == 0.0 ? 0.0 : fmin(ea * sup_deriv(O_CBRT, ad, ea), 1.5874010519681994 * cbrt(ea));
                se[h] = fn_bound(O_CBRT, xm, D, sd[h], u, rf);
                break;
            }
            default:   /* sin, cos, tan, exp, tanh, atan */
                se[h] = fn_bound(op, xm, ea == 0.0 ? 0.0 : ea * sup_deriv(op, ad, ea), sd[h], u, rf);
                break;
            }
            h++;
        }
        /* float32 overflow is a threshold too: a value whose bound reaches
         * FLT_MAX may be infinite on one side and finite on the other */
        if (h > 0 && se[h - 1] > 0.0 && fabs(sd[h - 1]) + se[h - 1] >= (double)FLT_MAX
            && fabs(sd[h - 1]) - se[h - 1] <= (double)FLT_MAX)
            near = 1;
    }
    *v32 = sf[0]; *v64 = sd[0]; *Eout = se[0]; *flip_out = flip; *near_out = near;
}

/* Per-row program outputs out[p*n_rows + r] for rows [0, n_rows) of a
 * feature-major dataset X[f*ld + r] (Sec. III: column-major data resident in
 * memory).  Programs are stored flat: program p is nodes[prog_off[p] ..
 * prog_off[p+1]) with constants consts[const_off[p] ..). */
void orc_evaluate_f32(const uint32_t *nodes, const int64_t *prog_off,
                      const float *consts, const int64_t *const_off, int32_t n_programs,
                      const float *X, int64_t ld, int64_t n_rows, float *out, int n_threads)
{
    (void)n_threads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
    for (int32_t p = 0; p < n_programs; ++p) {
        const uint32_t *pn = nodes + prog_off[p];
        int64_t len = prog_off[p + 1] - prog_off[p];
        const float *pc = consts + const_off[p];
        for (int64_t r = 0; r < n_rows; ++r)
            out[(int64_t)p * n_rows + r] = eval_row_f32(pn, len, pc, X, ld, r);
    }
}

void orc_evaluate_f64(const uint32_t *nodes, const int64_t *prog_off,
                      const float *consts, const int64_t *const_off, int32_t n_programs,
                      const float *X, int64_t ld, int64_t n_rows, double *out, int n_threads)
{
    (void)n_threads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
    for (int32_t p = 0; p < n_programs; ++p) {
        const uint32_t *pn = nodes + prog_off[p];
        int64_t len = prog_off[p + 1] - prog_off[p];
        const float *pc = consts + const_off[p];
        for (int64_t r = 0; r < n_rows; ++r)
            out[(int64_t)p * n_rows + r] = eval_row_f64(pn, len, pc, X, ld, r);
    }
}

/* Evaluate a subset of (program, row) pairs: out32[i], out64[i], the
 * conditioning bound ebound[i] (row_analysis with allowance u) and flags
 * flags[i] (bit 0: float32/float64 predicate flip, bit 1: predicate within
 * its bound of the threshold) for pair (prog[i], row[i]). */
void orc_evaluate_pairs(const uint32_t *nodes, const int64_t *prog_off,
                        const float *consts, const int64_t *const_off,
                        const float *X, int64_t ld,
                        const int32_t *prog, const int64_t *row, int64_t n_pairs, double u, double rf,
                        uint32_t exact_mask, float *out32, double *out64, double *ebound, uint8_t *flags, int n_threads)
{
    (void)n_threads;
#pragma omp parallel for schedule(static) num_threads(n_threads > 0 ? n_threads : 1)
    for (int64_t i = 0; i < n_pairs; ++i) {
        int32_t p = prog[i];
        const uint32_t *pn = nodes + prog_off[p];
        int64_t len = prog_off[p + 1] - prog_off[p];
        const float *pc = consts + const_off[p];
        int flip, near;
        row_analysis(pn, len, pc, X, ld, row[i], u, rf, exact_mask, &out32[i], &out64[i], &ebound[i], &flip,
                     &near);
        flags[i] = (uint8_t)(flip | (near << 1));
    }
}

/* ------------------------------------------------------------------------ */
/* Fitness (Sec. III-C3, the fitness metric computation step: a row-wise loss */
/* against the broadcast target, then a weighted sum per program).  Metrics:  */
/*   0 MAE  = sum w|yhat-y| / sum w                                           */
/*   1 MSE  = sum w (yhat-y)^2 / sum w                                        */
/*   2 RMSE = sqrt(MSE)                                                       */
/*   3 logistic loss (binary): yhat is a logit, l = log(1+e^yhat) - y*yhat,   */
/*     written in the overflow-free form max(z,0) - y z + log1p(e^-|z|)       */
/*   4 Pearson: |r| of the weighted correlation of yhat and y (0 when either  */
/*     weighted variance is zero or not finite)                               */
/* w == NULL means unit weights.                                              */
/*                                                                            */
/* Precision (reading): the program output yhat is the float32 stack value;   */
/* the row loss of MAE/MSE/RMSE/Pearson is formed in float64 from the float32 */
/* yhat, y, w; the logistic row loss is formed in float32 (it needs exp and   */
/* log1p); every sum over rows is accumulated in float64.  fit_f32path gets   */
/* this value; fit_f64 gets the same metric with yhat from the float64 stack  */
/* evaluation and every step in float64 (error reporting only).               */
/* ------------------------------------------------------------------------ */
/* ---- Spearman (Sec. III-C3): Pearson correlation of the rank vectors ---- */
/* Readings: rank 1 is the smallest value; tied values share the mean of the  */
/* ranks they span (the standard definition); ranks ignore the weights, and   */
/* the correlation of the ranks is the weighted Pearson of metric 4 (|r|,     */
/* 0 for a constant rank vector); NaN has no rank, so a NaN value, or a NaN   */
/* in the target, makes the fitness NaN.                                      */
static void merge_sort_idx(const double *v, int64_t *idx, int64_t *tmp, int64_t n)
{
    /* bottom-up merge sort of the indices by value (stable) */
    for (int64_t width = 1; width < n; width *= 2) {
        for (int64_t lo = 0; lo < n; lo += 2 * width) {
            int64_t mid = lo + width < n ? lo + width : n;
            int64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            int64_t i = lo, j = mid, k = lo;
            while (i < mid && j < hi) tmp[k++] = (v[idx[j]] < v[idx[i]]) ? idx[j++] : idx[i++];
            while (i < mid) tmp[k++] = idx[i++];
            while (j < hi) tmp[k++] = idx[j++];
        }
        memcpy(idx, tmp, sizeof(int64_t) * (size_t)n);
    }
}

/* average ranks (1-based) of v[0..n) into rank[]; idx receives the sort order */
static void average_ranks(const double *v, int64_t n, double *rank, int64_t *idx)
{
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t r = 0; r < n; ++r) idx[r] = r;
    merge_sort_idx(v, idx, tmp, n);
    free(tmp);
    int64_t i = 0;
    while (i < n) {
        int64_t j = i + 1;
        while (j < n && v[idx[j]] == v[idx[i]]) ++j;
        double avg = 0.5 * ((double)(i + 1) + (double)j);   /* mean of ranks i+1 .. j */
        for (int64_t k = i; k < j; ++k) rank[idx[k]] = avg;
        i = j;
    }
}

/* |weighted Pearson| of two float64 columns (0 for a constant column) */
static double pearson_abs(const double *av_in, const double *bv_in, const float *w, int64_t n)
{
    double sw = 0.0, ma = 0.0, mb = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        double wr = w ? (double)w[r] : 1.0;
        sw += wr; ma += wr * av_in[r]; mb += wr * bv_in[r];
    }
    ma /= sw; mb /= sw;
    double va = 0.0, vb = 0.0, cab = 0.0;
    /* a column that takes one value on every weighted row has variance 0
     * exactly, whatever rounding does to its computed mean */
    int const_a = 1, const_b = 1, seen = 0;
    double a0 = 0.0, b0 = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        double wr = w ? (double)w[r] : 1.0;
        double av = av_in[r], bv = bv_in[r];
        if (wr != 0.0) {
            if (!seen) { a0 = av; b0 = bv; seen = 1; }
            if (!(av == a0)) const_a = 0;
            if (!(bv == b0)) const_b = 0;
        }
        double a = av - ma;
        double b = bv - mb;
        va += wr * a * a; vb += wr * b * b; cab += wr * a * b;
    }
    if (const_a || const_b) return 0.0;
    if (!(va > 0.0) || !(vb > 0.0) || !isfinite(va) || !isfinite(vb)) return 0.0;
    return fabs(cab / sqrt(va * vb));
}

static double spearman_abs(const float *yh32, const double *yh64, const float *y, const float *w, int64_t n)
{
    double *a = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *b = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *ra = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *rb = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int has_nan = 0;
    for (int64_t r = 0; r < n; ++r) {
        a[r] = yh32 ? (double)yh32[r] : yh64[r];
        b[r] = (double)y[r];
        if (isnan(a[r]) || isnan(b[r])) has_nan = 1;
    }
    double out = NAN;
    if (!has_nan) {
        average_ranks(a, n, ra, idx);
        average_ranks(b, n, rb, idx);
        out = pearson_abs(ra, rb, w, n);
    }
    free(a); free(b); free(ra); free(rb); free(idx);
    return out;
}

static double metric_from_values(int metric, const float *yh32, const double *yh64,
                                 const float *y, const float *w, int64_t n)
{
    double sw = 0.0, s = 0.0;
    if (metric == 5) return spearman_abs(yh32, yh64, y, w, n);
    if (metric == 4) {
        double ma = 0.0, mb = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            double wr = w ? (double)w[r] : 1.0;
            double a = yh32 ? (double)yh32[r] : yh64[r];
            sw += wr; ma += wr * a; mb += wr * (double)y[r];
        }
        ma /= sw; mb /= sw;
        double va = 0.0, vb = 0.0, cab = 0.0;
        /* a column that takes one value on every weighted row has variance 0
         * exactly, whatever rounding does to its computed mean */
        int const_a = 1, const_b = 1, seen = 0;
        double a0 = 0.0, b0 = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            double wr = w ? (double)w[r] : 1.0;
            double av = yh32 ? (double)yh32[r] : yh64[r];
            double bv = (double)y[r];
            if (wr != 0.0) {
                if (!seen) { a0 = av; b0 = bv; seen = 1; }
                if (!(av == a0)) const_a = 0;
                if (!(bv == b0)) const_b = 0;
            }
            double a = av - ma;
            double b = bv - mb;
            va += wr * a * a; vb += wr * b * b; cab += wr * a * b;
        }
        if (const_a || const_b) return 0.0;
        if (!(va > 0.0) || !(vb > 0.0) || !isfinite(va) || !isfinite(vb)) return 0.0;
        return fabs(cab / sqrt(va * vb));
    }
    for (int64_t r = 0; r < n; ++r) {
        double wr = w ? (double)w[r] : 1.0;
        double l;
        if (metric == 3) {
            if (yh32) {
                float z = yh32[r], yr = y[r];
                float t1 = fmaxf(z, 0.0f);
                float t2 = yr * z;
                float t3 = t1 - t2;
                float t5 = log1pf(expf(-fabsf(z)));
                l = (double)(t3 + t5);
            } else {
                double z = yh64[r], yr = (double)y[r];
                l = fmax(z, 0.0) - yr * z + log1p(exp(-fabs(z)));
            }
        } else if (metric >= 6 && metric <= 9) {
            /* user loss i: U_i(yhat, y), U_i the two-argument user function
             * O_USER2 + i, in float32 (float32 path) or float64 */
            int uop = O_USER2 + (metric - 6);
            l = yh32 ? (double)user_f32(uop, yh32[r], y[r]) : user_f64(uop, yh64[r], (double)y[r]);
        } else {
            double d = (yh32 ? (double)yh32[r] : yh64[r]) - (double)y[r];
            l = (metric == 0) ? fabs(d) : d * d;
        }
        sw += wr;
        s += wr * l;
    }
    double m = s / sw;
    if (metric == 2) m = sqrt(m);
    return m;
}

/* First-order bound on how far the float32-path fitness can move when each
 * row's float32 output moves by at most its row_analysis bound E[r]:
 * sum_r |d fitness / d yhat_r| E[r] (plus the second-order term of MSE). */
/* Spearman's sensitivity.  Every value may sit anywhere in [v - E, v + E]  */
/* on the other side; rows whose intervals form one connected component of    */
/* the (strict) overlap graph may be reordered or tied among themselves,      */
/* while different components keep their order, so a row of a component of   */
/* m rows changes rank by at most d = m - 1.  With a, b the centred value and */
/* target ranks: the cross term moves by at most sum w |b| d exactly (b sums  */
/* to zero under w), and the value ranks' weighted norm by at most            */
/* D = sqrt(sum w d'^2), d' = d + (sum w d) / W (the shift of their mean);    */
/* |rho| then lies in [(|c| - DC) / ((sa + D) sb), (|c| + DC) / ((sa - D) sb)]. */
static double spearman_bound(const float *yh, const double *E, const float *y, const float *w, int64_t n,
                             double rho)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *lo = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *ra = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *rb = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int y_nan = 0;
    for (int64_t r = 0; r < n; ++r) {
        v[r] = (double)yh[r];
        lo[r] = v[r] - E[r];
        if (isnan(y[r])) y_nan = 1;
    }
    if (y_nan) {                            /* NaN on both sides, whatever the values */
        free(v); free(lo); free(ra); free(rb); free(d); free(idx);
        return 0.0;
    }
    average_ranks(lo, n, ra, idx);          /* idx: rows by ascending lower end */
    int64_t i = 0;
    while (i < n) {
        double hi = v[idx[i]] + E[idx[i]];
        int64_t j = i + 1;
        while (j < n && lo[idx[j]] < hi) {
            double h2 = v[idx[j]] + E[idx[j]];
            if (h2 > hi) hi = h2;
            ++j;
        }
        for (int64_t k = i; k < j; ++k) d[idx[k]] = (double)(j - i - 1);
        i = j;
    }
    average_ranks(v, n, ra, idx);
    for (int64_t r = 0; r < n; ++r) lo[r] = (double)y[r];
    average_ranks(lo, n, rb, idx);
    double W = 0.0, ma = 0.0, mb = 0.0, shift = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        double wr = w ? (double)w[r] : 1.0;
        W += wr; ma += wr * ra[r]; mb += wr * rb[r]; shift += wr * d[r];
    }
    ma /= W; mb /= W; shift /= W;
    double va = 0.0, vb = 0.0, cab = 0.0, dc = 0.0, dn = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        double wr = w ? (double)w[r] : 1.0;
        double a = ra[r] - ma, b = rb[r] - mb, dd = d[r] + shift;
        va += wr * a * a; vb += wr * b * b; cab += wr * a * b;
        dc += wr * fabs(b) * d[r];
        dn += wr * dd * dd;
    }
    free(v); free(lo); free(ra); free(rb); free(d); free(idx);
    (void)rho;
    if (!(vb > 0.0)) return 0.0;                      /* constant target: 0 on both sides */
    if (shift == 0.0) return 0.0;                     /* no component can reorder */
    double sa = sqrt(va), sb = sqrt(vb), D = sqrt(dn);
    double r0 = va > 0.0 ? fabs(cab) / (sa * sb) : 0.0;
    double rmax = (sa - D > 0.0) ? (fabs(cab) + dc) / ((sa - D) * sb) : 1.0;
    double rmin = (fabs(cab) - dc) / ((sa + D) * sb);
    if (rmax > 1.0) rmax = 1.0;
    if (rmin < 0.0) rmin = 0.0;
    double up = rmax - r0, down = r0 - rmin;
    return up > down ? up : down;
}

static double fitness_bound(int metric, const float *yh, const double *E, const float *y,
                            const float *w, int64_t n, double fit)
{
    if (metric == 5) return spearman_bound(yh, E, y, w, n, fit);
    double W = 0.0;
    for (int64_t r = 0; r < n; ++r) W += w ? (double)w[r] : 1.0;
    double B = 0.0;
    if (metric == 4) {
        /* r = c / (sa sb) with c = sum w a b, sa^2 = sum w a^2 over the
         * centred columns.  Rows moving by d_r, |d_r| <= E_r, give (b is
         * centred, so d's mean drops out of c)
         *   r' - r = (1/sa') sum w d (b/sb - k r a) - r |d_c|^2 / ((sa' + sa) sa'),
         * k = 2 / (sa' + sa), an identity; and sa'^2 = sa^2 + 2 sum w a d +
         * |d_c|^2 lies within [sa^2 - 2A, sa^2 + 2A + dn], A = sum w |a| E,
         * dn = sum w E^2.  Bounding sa' below by sa_lo and taking k at both
         * ends of its range row by row gives a bound on |r' - r| that tends
         * to the first-order sum w E |b/(sa sb) - r a/sa^2| as E -> 0.  A
         * column that may become constant (sa_lo = 0) may take any |r|: the
         * bound is then 1. */
        double ma = 0.0, mb = 0.0, va = 0.0, vb = 0.0, cab = 0.0, dn = 0.0, A = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            double wr = w ? (double)w[r] : 1.0;
            ma += wr * (double)yh[r]; mb += wr * (double)y[r];
        }
        ma /= W; mb /= W;
        for (int64_t r = 0; r < n; ++r) {
            double wr = w ? (double)w[r] : 1.0;
            double a = (double)yh[r] - ma, b = (double)y[r] - mb;
            va += wr * a * a; vb += wr * b * b; cab += wr * a * b;
            dn += mul0(wr, E[r] * E[r]);
            A += mul0(wr * fabs(a), E[r]);
        }
        if (!(vb > 0.0)) return 0.0;                 /* constant target: 0 on both sides */
        if (!(dn > 0.0)) return 0.0;                 /* no row can move */
        if (!isfinite(va) || !isfinite(dn) || !isfinite(A)) return INFINITY;
        double lo2 = va - 2.0 * A;
        if (!(lo2 > 0.0)) return 1.0;
        double sa = sqrt(va), sb = sqrt(vb), sa_lo = sqrt(lo2), sa_hi = sqrt(va + 2.0 * A + dn);
        double rr = cab / (sa * sb);
        double k1 = 2.0 / (sa + sa_hi), k2 = 2.0 / (sa + sa_lo);
        double S = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            double wr = w ? (double)w[r] : 1.0;
            double a = (double)yh[r] - ma, b = (double)y[r] - mb;
            double g1 = fabs(b / sb - k1 * rr * a), g2 = fabs(b / sb - k2 * rr * a);
            S += mul0(wr * (g1 > g2 ? g1 : g2), E[r]);
        }
        double bound = S / sa_lo + fabs(rr) * dn / ((sa_lo + sa) * sa_lo);
        return bound < 1.0 ? bound : 1.0;
    }
    for (int64_t r = 0; r < n; ++r) {
        double wr = w ? (double)w[r] : 1.0;
        double d = (double)yh[r] - (double)y[r];
        if (metric == 0 || metric == 3) B += mul0(wr, E[r]);
        else B += mul0(2.0 * wr * fabs(d), E[r]) + mul0(wr, E[r] * E[r]);
    }
    B /= W;
    if (metric == 2) B = fit > 0.0 ? B / (2.0 * fit) : sqrt(B);
    return B;
}

void orc_fitness(const uint32_t *nodes, const int64_t *prog_off,
                 const float *consts, const int64_t *const_off, int32_t n_programs,
                 const float *X, int64_t ld, int64_t n_rows,
                 const float *y, const float *w, int32_t metric,
                 double *fit_f32path, double *fit_f64, double u, double rf, uint32_t exact_mask,
                 double *fbound, int32_t *fnear, int n_threads)
{
    (void)n_threads;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        size_t nn = (size_t)(n_rows > 0 ? n_rows : 1);
        float *yh32 = (float *)malloc(nn * sizeof(float));
        double *yh64 = (fit_f64 || fbound) ? (double *)malloc(nn * sizeof(double)) : NULL;
        double *E = fbound ? (double *)malloc(nn * sizeof(double)) : NULL;
#pragma omp for schedule(dynamic, 1)
        for (int32_t p = 0; p < n_programs; ++p) {
            const uint32_t *pn = nodes + prog_off[p];
            int64_t len = prog_off[p + 1] - prog_off[p];
            const float *pc = consts + const_off[p];
            int32_t nnear = 0;
            if (fbound) {
                for (int64_t r = 0; r < n_rows; ++r) {
                    int flip, near;
                    row_analysis(pn, len, pc, X, ld, r, u, rf, exact_mask, &yh32[r], &yh64[r], &E[r], &flip,
                                 &near);
                    nnear += near;
                }
            } else {
                for (int64_t r = 0; r < n_rows; ++r)
                    yh32[r] = eval_row_f32(pn, len, pc, X, ld, r);
                if (fit_f64)
                    for (int64_t r = 0; r < n_rows; ++r)
                        yh64[r] = eval_row_f64(pn, len, pc, X, ld, r);
            }
            fit_f32path[p] = metric_from_values(metric, yh32, NULL, y, w, n_rows);
            if (fit_f64) fit_f64[p] = metric_from_values(metric, NULL, yh64, y, w, n_rows);
            if (fbound) {
                fbound[p] = fitness_bound(metric, yh32, E, y, w, n_rows, fit_f32path[p]);
                if (fnear) fnear[p] = nnear;
            }
        }
        free(yh32);
        free(yh64);
        free(E);
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), the counter-based       */
/* generator the paper uses for tournament draws (Sec. III-B).  Round:        */
/* (hi0,lo0) = M0*x0, (hi1,lo1) = M1*x2; out = (hi1^x1^k0, lo1, hi0^x3^k1,     */
/* lo0); the key is bumped by the Weyl constants between rounds.              */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        x0 = n0; x1 = lo1; x2 = n2; x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream map (reading): key = (seed low word, seed high word); counter =
 * (block j, item i, generation g, stream tag s).  Draw d of an item is word
 * (d mod 4) of block floor(d/4).  Stream tags: 0 tournament, 1 init. */
typedef struct { uint64_t seed; uint32_t item, gen, tag; uint32_t d; uint32_t buf[4]; uint32_t have_block; } orc_rng;

static void rng_init(orc_rng *g, uint64_t seed, uint32_t item, uint32_t gen, uint32_t tag)
{
    g->seed = seed; g->item = item; g->gen = gen; g->tag = tag; g->d = 0; g->have_block = 0xffffffffu;
}

static uint32_t rng_word(orc_rng *g)
{
    uint32_t block = g->d / 4u, lane = g->d % 4u;
    if (g->have_block != block) {
        uint32_t ctr[4] = {block, g->item, g->gen, g->tag};
        uint32_t key[2] = {(uint32_t)(g->seed & 0xffffffffu), (uint32_t)(g->seed >> 32)};
        orc_philox4x32_10(ctr, key, g->buf);
        g->have_block = block;
    }
    g->d++;
    return g->buf[lane];
}

/* uniform integer in [0, n): floor(w * n / 2^32) */
static uint32_t word_below(uint32_t w, uint32_t n) { return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32); }
/* uniform float in [0, 1): top 24 bits of the word times 2^-24 */
static float word_unit(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

/* Raw draw access for tests: words d0 .. d0+n-1 of (seed, item, gen, tag). */
void orc_philox_words(uint64_t seed, uint32_t item, uint32_t gen, uint32_t tag,
                      uint32_t d0, uint32_t n, uint32_t *out)
{
    orc_rng g;
    rng_init(&g, seed, item, gen, tag);
    g.d = d0;
    for (uint32_t i = 0; i < n; ++i) out[i] = rng_word(&g);
}

/* ------------------------------------------------------------------------ */
/* Tournament selection (Sec. III-C1): tournament t draws k program indices,  */
/* with replacement, and keeps the one with the best adjusted fitness         */
/*   fitness = raw + c*len  (criterion favouring smaller values, Eqs.         */
/*   (parsimony), (fitness)); for a criterion favouring larger values the     */
/*   penalty is subtracted and the largest wins.                              */
/* Readings: float32 arithmetic, each op rounded (no fused multiply-add);     */
/* strict comparison so the earliest draw wins ties; NaN ranks worst.         */
/* ------------------------------------------------------------------------ */
void orc_tournament(const float *fitness, const int32_t *len, int32_t n_programs,
                    int32_t larger_is_better, float parsimony, int32_t k,
                    int32_t n_tournaments, uint64_t seed, uint64_t generation,
                    int32_t *winners)
{
    for (int32_t t = 0; t < n_tournaments; ++t) {
        orc_rng g;
        rng_init(&g, seed, (uint32_t)t, (uint32_t)generation, 0u);
        int32_t best = -1;
        float best_adj = 0.0f;
        for (int32_t d = 0; d < k; ++d) {
            int32_t idx = (int32_t)word_below(rng_word(&g), (uint32_t)n_programs);
            volatile float pen = parsimony * (float)len[idx];
            float adj = larger_is_better ? fitness[idx] - pen : fitness[idx] + pen;
            int take;
            if (best < 0) take = 1;
            else if (isnan(adj)) take = 0;
            else if (isnan(best_adj)) take = 1;
            else take = larger_is_better ? (adj > best_adj) : (adj < best_adj);
            if (take) { best = idx; best_adj = adj; }
        }
        winners[t] = best;
    }
}

/* Indices drawn by tournament t, for tests (draw d -> index). */
void orc_tournament_draws(int32_t n_programs, int32_t k, int32_t t, uint64_t seed,
                          uint64_t generation, int32_t *idx_out)
{
    orc_rng g;
    rng_init(&g, seed, (uint32_t)t, (uint32_t)generation, 0u);
    for (int32_t d = 0; d < k; ++d)
        idx_out[d] = (int32_t)word_below(rng_word(&g), (uint32_t)n_programs);
}

/* ------------------------------------------------------------------------ */
/* Program generation (Sec. II-A: Full, Grow, ramped half-and-half; Sec.      */
/* III-A: prefix lists are produced directly).  Readings, all draws from the  */
/* init stream (tag 1), item = program index, generation 0, one word per      */
/* decision taken in prefix (pre-)order:                                      */
/*  RHH: word -> Grow if unit < 0.5 else Full; word -> depth d in            */
/*       [min_depth, max_depth].  Node at depth k: k == d -> terminal;        */
/*       k == 0 < d -> function; 0 < k < d -> Full: function, Grow: one of    */
/*       (functions, features, constant) uniformly.  Terminal: one of         */
/*       (features, constant) uniformly.  A constant takes one more word:      */
/*       lo + (hi-lo)*unit in float32.  Constants are unavailable when        */
/*       lo > hi or once max_consts (> 0) of them are used.                   */
/*  EXACT_LEN: word -> L in [min_len, max_len]; positions L-1 .. 0 are filled */
/*       right to left with stack height h; allowed at position i:            */
/*       terminal if h+1 <= 20 and h <= i; unary if h >= 1 and h-1 <= i;      */
/*       binary if h >= 2 and h-2 <= i; (plus a parity rule when there is no  */
/*       unary function).  One word picks uniformly among the allowed items,  */
/*       listed as features, constant, unary ops, binary ops.                 */
/* Function set: bit (1 << opcode) of fmask for opcodes 2..22 and 24..31.     */
/* Constant slots are numbered 0,1,.. in prefix order.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t *nodes; int64_t n, cap;
    float *consts; int64_t nc, ccap;
    int overflow;
} orc_buf;

static void put_node(orc_buf *b, uint32_t w)
{
    if (b->nodes && b->n < b->cap) b->nodes[b->n] = w; else if (b->nodes) b->overflow = 1;
    b->n++;
}
static void put_const(orc_buf *b, float v)
{
    if (b->consts && b->nc < b->ccap) b->consts[b->nc] = v; else if (b->consts) b->overflow = 1;
    b->nc++;
}

typedef struct {
    int n_features;
    int funcs[O_LIMIT]; int n_funcs;    /* enabled functions in opcode order */
    int un[O_LIMIT]; int n_un;
    int bin[O_LIMIT]; int n_bin;
    float lo, hi; int consts_on; int max_consts;
} orc_gen_cfg;

static float draw_const(orc_rng *g, const orc_gen_cfg *cfg)
{
    float u = word_unit(rng_word(g));
    float span = cfg->hi - cfg->lo;
    float t = span * u;
    return cfg->lo + t;
}

/* recursive pre-order builder for Full / Grow */
static void grow_node(orc_rng *g, const orc_gen_cfg *cfg, orc_buf *b, int depth, int target,
                      int full, int64_t *n_consts_used)
{
    int const_ok = cfg->consts_on && (cfg->max_consts <= 0 || *n_consts_used < cfg->max_consts);
    int n_term = cfg->n_features + (const_ok ? 1 : 0);
    int is_func;
    int pick;
    if (depth == target) {
        is_func = 0;
        pick = (int)word_below(rng_word(g), (uint32_t)n_term);
    } else if (depth == 0 || full) {
        is_func = 1;
        pick = (int)word_below(rng_word(g), (uint32_t)cfg->n_funcs);
    } else {
        pick = (int)word_below(rng_word(g), (uint32_t)(cfg->n_funcs + n_term));
        if (pick < cfg->n_funcs) is_func = 1;
        else { is_func = 0; pick -= cfg->n_funcs; }
    }
    if (is_func) {
        int op = cfg->funcs[pick];
        put_node(b, (uint32_t)op);
        for (int a = 0; a < op_arity(op); ++a)
            grow_node(g, cfg, b, depth + 1, target, full, n_consts_used);
    } else if (pick < cfg->n_features) {
        put_node(b, (uint32_t)O_VAR | ((uint32_t)pick << 8));
    } else {
        put_node(b, (uint32_t)O_CONST | ((uint32_t)(*n_consts_used) << 8));
        put_const(b, draw_const(g, cfg));
        (*n_consts_used)++;
    }
}

static int gen_exact(orc_rng *g, const orc_gen_cfg *cfg, orc_buf *b, int min_len, int max_len)
{
    int L = min_len + (int)word_below(rng_word(g), (uint32_t)(max_len - min_len + 1));
    if (cfg->n_un == 0 && (L % 2) == 0) {
        if (L - 1 >= min_len && L - 1 >= 1) L -= 1; else L += 1;
    }
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)L);
    float *cv = (float *)malloc(sizeof(float) * (size_t)L);
    int nconst = 0;
    int h = 0;
    for (int i = L - 1; i >= 0; --i) {
        int const_ok = cfg->consts_on && (cfg->max_consts <= 0 || nconst < cfg->max_consts);
        int n_term = cfg->n_features + (const_ok ? 1 : 0);
        int t_ok = (h + 1 <= ORC_STACK) && (h <= i);
        int u_ok = (cfg->n_un > 0) && (h >= 1) && (h - 1 <= i);
        int b_ok = (cfg->n_bin > 0) && (h >= 2) && (h - 2 <= i);
        if (cfg->n_un == 0) {
            /* with only +1 / -1 steps, the height after this position and the
             * number of positions left must have opposite parity (end at 1) */
            if (t_ok && (((h + 1) - 1 + i) % 2 != 0)) t_ok = 0;
            if (b_ok && (((h - 1) - 1 + i) % 2 != 0)) b_ok = 0;
        }
        int nt = t_ok ? n_term : 0, nu = u_ok ? cfg->n_un : 0, nb = b_ok ? cfg->n_bin : 0;
        int tot = nt + nu + nb;
        if (tot == 0) { free(tmp); free(cv); return -1; }
        int pick = (int)word_below(rng_word(g), (uint32_t)tot);
        if (pick < nt) {
            if (pick < cfg->n_features) tmp[i] = (uint32_t)O_VAR | ((uint32_t)pick << 8);
            else { tmp[i] = (uint32_t)O_CONST; cv[i] = draw_const(g, cfg); nconst++; }
            h += 1;
        } else if (pick < nt + nu) {
            tmp[i] = (uint32_t)cfg->un[pick - nt];
        } else {
            tmp[i] = (uint32_t)cfg->bin[pick - nt - nu];
            h -= 1;
        }
    }
    int slot = 0;
    for (int i = 0; i < L; ++i) {
        if ((tmp[i] & 0xffu) == O_CONST) {
            put_node(b, (uint32_t)O_CONST | ((uint32_t)slot << 8));
            put_const(b, cv[i]);
            slot++;
        } else {
            put_node(b, tmp[i]);
        }
    }
    free(tmp);
    free(cv);
    return 0;
}

/* one program by the method: 0 RHH, 1 FULL, 2 GROW, 3 EXACT_LEN */
static int gen_one(orc_rng *g, const orc_gen_cfg *cfg, orc_buf *b, int method, int min_depth,
                   int max_depth, int min_len, int max_len)
{
    if (method == 3) return gen_exact(g, cfg, b, min_len, max_len);
    int full;
    if (method == 0) full = !(word_unit(rng_word(g)) < 0.5f);
    else full = (method == 1);
    int depth = min_depth + (int)word_below(rng_word(g), (uint32_t)(max_depth - min_depth + 1));
    int64_t used = 0;
    grow_node(g, cfg, b, 0, depth, full, &used);
    return 0;
}

static int fill_cfg(orc_gen_cfg *cfg, int32_t n_features, uint32_t fmask, float const_lo,
                    float const_hi, int32_t max_consts)
{
    memset(cfg, 0, sizeof *cfg);
    if (n_features < 1) return -1;
    if (fmask & (1u << 23 | 3u)) return -1;
    cfg->n_features = n_features;
    for (int op = O_ADD; op < O_LIMIT; ++op) {
        if (op_arity(op) > 0 && (fmask & (1u << op))) {
            cfg->funcs[cfg->n_funcs++] = op;
            if (op_arity(op) == 1) cfg->un[cfg->n_un++] = op; else cfg->bin[cfg->n_bin++] = op;
        }
    }
    if (cfg->n_funcs == 0) return -1;
    cfg->lo = const_lo; cfg->hi = const_hi;
    cfg->consts_on = !(const_lo > const_hi);
    cfg->max_consts = max_consts;
    return 0;
}

/* method: 0 RHH, 1 FULL, 2 GROW, 3 EXACT_LEN.  Buffers may be NULL (sizes
 * only).  Returns 0 on success, -1 bad arguments, -2 a buffer is too small. */
int orc_build_population(int32_t n_programs, int32_t n_features, int32_t method,
                         int32_t min_depth, int32_t max_depth, int32_t min_len, int32_t max_len,
                         uint32_t fmask, float const_lo, float const_hi, int32_t max_consts,
                         uint64_t seed,
                         uint32_t *nodes, int64_t nodes_cap, int64_t *prog_off,
                         float *consts, int64_t consts_cap, int64_t *const_off, int32_t *len,
                         int64_t *total_nodes, int64_t *total_consts)
{
    orc_gen_cfg cfg;
    memset(&cfg, 0, sizeof cfg);
    if (n_programs < 0 || n_features < 1) return -1;
    cfg.n_features = n_features;
    for (int op = O_ADD; op < O_LIMIT; ++op) {
        if (op_arity(op) > 0 && (fmask & (1u << op))) {
            cfg.funcs[cfg.n_funcs++] = op;
            if (op_arity(op) == 1) cfg.un[cfg.n_un++] = op; else cfg.bin[cfg.n_bin++] = op;
        }
    }
    if (fmask & (1u << 23 | 3u)) return -1;
    if (cfg.n_funcs == 0) return -1;
    cfg.lo = const_lo; cfg.hi = const_hi;
    cfg.consts_on = !(const_lo > const_hi);
    cfg.max_consts = max_consts;
    if (method == 3) {
        if (min_len < 1 || max_len < min_len) return -1;
        if (cfg.n_bin == 0 && max_len > 1) return -1;
    } else if (method >= 0 && method <= 2) {
        if (min_depth < 0 || max_depth < min_depth || max_depth > ORC_STACK - 1) return -1;
    } else {
        return -1;
    }
    orc_buf b;
    b.nodes = nodes; b.n = 0; b.cap = nodes_cap;
    b.consts = consts; b.nc = 0; b.ccap = consts_cap; b.overflow = 0;
    for (int32_t p = 0; p < n_programs; ++p) {
        orc_rng g;
        rng_init(&g, seed, (uint32_t)p, 0u, 1u);
        int64_t n0 = b.n, c0 = b.nc;
        if (prog_off && nodes) prog_off[p] = n0;
        if (const_off && nodes) const_off[p] = c0;
        if (gen_one(&g, &cfg, &b, method, min_depth, max_depth, min_len, max_len) != 0) return -1;
        if (len && nodes) len[p] = (int32_t)(b.n - n0);
    }
    if (prog_off && nodes) prog_off[n_programs] = b.n;
    if (const_off && nodes) const_off[n_programs] = b.nc;
    if (total_nodes) *total_nodes = b.n;
    if (total_consts) *total_consts = b.nc;
    return b.overflow ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Reverse-mode derivative of fitness with respect to every program constant, */
/* in float64 (not in the paper).  For each row the program is evaluated in   */
/* float64 keeping every node's value; the adjoint of the root is the         */
/* derivative of the metric with respect to that row's output; nodes are then */
/* visited parent-before-child (prefix order), handing each child its share    */
/* by the local partial derivatives (readings):                               */
/*   add (1,1); sub (1,-1); mul (b,a); pdiv (1/b, -a/b^2) if |b|>eps else 0;  */
/*   plog 1/a if |a|>eps else 0; psqrt sign(a)/(2 sqrt|a|), 0 at a = 0;       */
/*   sin cos a; cos -sin a; tan 1 + tan^2 a; neg -1; max / min 1 for the      */
/*   operand selected (the first on ties), 0 for the other; atan2(a, b)       */
/*   (b, -a)/(a^2+b^2), 0 at the origin; abs sign(a) (0 at 0); exp exp(a);    */
/*   inv -1/a^2 if |a|>eps else 0; sq 2a; cube 3a^2; tanh 1 - tanh^2 a;       */
/*   atan 1/(1+a^2); cbrt 1/(3 cbrt(a)^2), 0 at a = 0.                        */
/* Seeds: MSE 2w(yh-y)/W; MAE w sign(yh-y)/W; RMSE dMSE/(2 RMSE) (0 if RMSE   */
/* is 0); logistic w(sigmoid(yh)-y)/W; Pearson d|r|/dyh.                      */
/* grad[const_off[p] + s] receives gscale[p] * d fitness_p / d c_s.           */
/* With f32_tape the forward pass is the float32 evaluation and the sweep     */
/* takes its partials, in float64, at those float32 values: the derivative    */
/* of the float32 program, whose protected branches and values are the ones   */
/* a float32 evaluation takes (reading; with mc_u > 0 only the sweep's        */
/* partials and seed are perturbed then).                                     */
/* Any program length: the per-thread buffers take the longest program.      */
/* ------------------------------------------------------------------------ */
static double local_partial(int op, int which, double a, double b, double out)
{
    switch (op) {
    case O_ADD: return 1.0;
    case O_SUB: return which == 0 ? 1.0 : -1.0;
    case O_MUL: return which == 0 ? b : a;
    case O_DIV:
        if (!(fabs(b) > (double)ORC_EPS)) return 0.0;
        return which == 0 ? 1.0 / b : -a / (b * b);
    case O_NEG: return -1.0;
    case O_LOG: return fabs(a) > (double)ORC_EPS ? 1.0 / a : 0.0;
    case O_SQRT:
        if (a == 0.0) return 0.0;
        return (a > 0.0 ? 1.0 : -1.0) / (2.0 * sqrt(fabs(a)));
    case O_SIN: return cos(a);
    case O_COS: return -sin(a);
    case O_TAN: return 1.0 + out * out;
    case O_MAX: {   /* the selected operand carries the derivative */
        int first = (a >= b) || isnan(b);
        return which == 0 ? (first ? 1.0 : 0.0) : (first ? 0.0 : 1.0);
    }
    case O_MIN: {
        int first = (a <= b) || isnan(b);
        return which == 0 ? (first ? 1.0 : 0.0) : (first ? 0.0 : 1.0);
    }
    case O_ATAN2: {
        double r2 = a * a + b * b;
        if (!(r2 > 0.0)) return 0.0;
        return which == 0 ? b / r2 : -a / r2;
    }
    case O_ABS: return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0);
    case O_EXP: return out;
    case O_INV: return fabs(a) > (double)ORC_EPS ? -out * out : 0.0;
    case O_SQ: return 2.0 * a;
    case O_CUBE: return 3.0 * a * a;
    case O_TANH: return 1.0 - out * out;
    case O_ATAN: return 1.0 / (1.0 + a * a);
    case O_CBRT: return out != 0.0 ? 1.0 / (3.0 * out * out) : 0.0;
    default: return 0.0;
    }
}

/* ---- Monte Carlo arithmetic (Parker, 1997), for conditioning estimates ---- */
/* With u > 0 every operation's result v is replaced by v (1 + s u), s = +-1,  */
/* the sign taken from SplitMix64 (Steele, Lea and Flood, 2014) of the         */
/* (seed, row, node, role) counter.  The spread of the derivatives over a few  */
/* seeds estimates how far float32 rounding (relative error u per operation)   */
/* can move them.  With u = 0 nothing is perturbed.                            */
static double mc_factor(double u, uint64_t seed, int64_t r, int64_t i, int role)
{
    if (u == 0.0) return 1.0;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull *
                 (1ull + (uint64_t)r * 16384ull + (uint64_t)i * 4ull + (uint64_t)role);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (z >> 63) ? 1.0 - u : 1.0 + u;
}

/* Forward pass of one row keeping every node's value val[i] and the end     */
/* (one past) of its subtree endi[i]; returns the program value.  In float64, */
/* or, with f32 set, the float32 evaluation (each node's float32 value,       */
/* widened: the point at which a float32 program's derivative is taken);      */
/* Monte Carlo perturbation applies to the float64 pass only.                 */
static double forward_row(const uint32_t *pn, int64_t L, const float *pc, const float *X,
                          int64_t ld, int64_t r, double u, uint64_t seed, int f32,
                          double *val, int64_t *endi)
{
    double st[ORC_STACK];
    int h = 0;
    for (int64_t i = L - 1; i >= 0; --i) {
        int op = (int)(pn[i] & 0xffu);
        uint32_t arg = pn[i] >> 8;
        int ar = op_arity(op);
        double v;
        if (ar == 0) {
            v = (op == O_VAR) ? (double)X[(int64_t)arg * ld + r] : (double)pc[arg];
            endi[i] = i + 1;
        } else if (ar == 1) {
            double a = st[--h];
            v = f32 ? (double)op_f32(op, (float)a, 0.0f) : op_f64(op, a, 0.0) * mc_factor(u, seed, r, i, 0);
            endi[i] = endi[i + 1];
        } else {
            double a = st[--h];
            double b = st[--h];
            v = f32 ? (double)op_f32(op, (float)a, (float)b) : op_f64(op, a, b) * mc_factor(u, seed, r, i, 0);
            endi[i] = endi[endi[i + 1]];
        }
        val[i] = v;
        st[h++] = v;
    }
    return val[0];
}


void orc_grad_consts(const uint32_t *nodes, const int64_t *prog_off,
                     const float *consts, const int64_t *const_off, int32_t n_programs,
                     const float *X, int64_t ld, int64_t n_rows,
                     const float *y, const float *w, int32_t metric,
                     const double *gscale, double *grad, double *fit_out,
                     double mc_u, uint64_t mc_seed, int f32_tape, int n_threads)
{
    /* per-thread buffers for the longest program (any length) */
    int64_t max_len = 1;
    for (int32_t p = 0; p < n_programs; ++p)
        if (prog_off[p + 1] - prog_off[p] > max_len) max_len = prog_off[p + 1] - prog_off[p];
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        double *yh = (double *)malloc(sizeof(double) * (size_t)(n_rows > 0 ? n_rows : 1));
        double *val = (double *)malloc(sizeof(double) * (size_t)(max_len + 1));
        double *adj = (double *)malloc(sizeof(double) * (size_t)(max_len + 1));
        int64_t *endi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(max_len + 1));
#pragma omp for schedule(dynamic, 1)
        for (int32_t p = 0; p < n_programs; ++p) {
            const uint32_t *pn = nodes + prog_off[p];
            int64_t L = prog_off[p + 1] - prog_off[p];
            const float *pc = consts + const_off[p];
            int64_t nc = const_off[p + 1] - const_off[p];
            double *gp = grad + const_off[p];
            for (int64_t s = 0; s < nc; ++s) gp[s] = 0.0;
            /* forward pass for the metric's global statistics */
            double W = 0.0, S = 0.0;
            for (int64_t r = 0; r < n_rows; ++r)
                yh[r] = f32_tape ? (double)eval_row_f32(pn, L, pc, X, ld, r)
                        : mc_u == 0.0 ? eval_row_f64(pn, L, pc, X, ld, r)
                                      : forward_row(pn, L, pc, X, ld, r, mc_u, mc_seed, 0, val, endi);
            double ma = 0.0, mb = 0.0, va = 0.0, vb = 0.0, cab = 0.0, rr = 0.0;
            for (int64_t r = 0; r < n_rows; ++r) {
                double wr = w ? (double)w[r] : 1.0;
                W += wr;
                if (metric == 0) S += wr * fabs(yh[r] - (double)y[r]);
                else if (metric == 1 || metric == 2) S += wr * (yh[r] - (double)y[r]) * (yh[r] - (double)y[r]);
                else if (metric == 3) {
                    double z = yh[r];
                    S += wr * (fmax(z, 0.0) - (double)y[r] * z + log1p(exp(-fabs(z))));
                }
                ma += wr * yh[r]; mb += wr * (double)y[r];
            }
            double fit;
            if (metric == 4) {
                ma /= W; mb /= W;
                for (int64_t r = 0; r < n_rows; ++r) {
                    double wr = w ? (double)w[r] : 1.0;
                    double a = yh[r] - ma, b = (double)y[r] - mb;
                    va += wr * a * a; vb += wr * b * b; cab += wr * a * b;
                }
                int ok = (va > 0.0) && (vb > 0.0) && isfinite(va) && isfinite(vb);
                rr = ok ? cab / sqrt(va * vb) : 0.0;
                fit = fabs(rr);
                if (!ok) { if (fit_out) fit_out[p] = 0.0; continue; }
            } else {
                fit = S / W;
                if (metric == 2) fit = sqrt(fit);
            }
            if (fit_out) fit_out[p] = fit;
            double gs = gscale ? gscale[p] : 1.0;
            if (nc == 0) continue;
            /* per-row reverse sweep */
            for (int64_t r = 0; r < n_rows; ++r) {
                double wr = w ? (double)w[r] : 1.0;
                double d = yh[r] - (double)y[r];
                double seed;
                switch (metric) {
                case 0: seed = wr * (d > 0 ? 1.0 : (d < 0 ? -1.0 : 0.0)) / W; break;
                case 1: seed = 2.0 * wr * d / W; break;
                case 2: seed = fit > 0.0 ? (2.0 * wr * d / W) / (2.0 * fit) : 0.0; break;
                case 3: seed = wr * (1.0 / (1.0 + exp(-yh[r])) - (double)y[r]) / W; break;
                default: {
                    double a = yh[r] - ma, b = (double)y[r] - mb;
                    double dr = wr * (b / sqrt(va * vb) - rr * a / va);
                    seed = (rr >= 0.0 ? 1.0 : -1.0) * dr;
                }
                }
                seed *= gs * mc_factor(mc_u, mc_seed, r, 0, 3);
                forward_row(pn, L, pc, X, ld, r, mc_u, mc_seed, f32_tape, val, endi);
                for (int64_t i = 0; i < L; ++i) adj[i] = 0.0;
                adj[0] = seed;
                for (int64_t i = 0; i < L; ++i) {
                    int op = (int)(pn[i] & 0xffu);
                    int ar = op_arity(op);
                    if (op == O_CONST) { gp[pn[i] >> 8] += adj[i]; continue; }
                    if (ar == 0 || adj[i] == 0.0) continue;
                    int64_t ia = i + 1;
                    if (ar == 1) {
                        adj[ia] += adj[i] * local_partial(op, 0, val[ia], 0.0, val[i])
                                   * mc_factor(mc_u, mc_seed, r, i, 1);
                    } else {
                        int64_t ib = endi[ia];
                        adj[ia] += adj[i] * local_partial(op, 0, val[ia], val[ib], val[i])
                                   * mc_factor(mc_u, mc_seed, r, i, 1);
                        adj[ib] += adj[i] * local_partial(op, 1, val[ia], val[ib], val[i])
                                   * mc_factor(mc_u, mc_seed, r, i, 2);
                    }
                }
            }
        }
        free(endi);
        free(adj);
        free(val);
        free(yh);
    }
}

/* ------------------------------------------------------------------------ */
/* Genetic operations (Sec. II-A lists reproduction, point, hoist, subtree  */
/* and crossover; Sec. III-C pre-draws each offspring's operation so the    */
/* number of tournaments is known; Sec. III-C2 hoists the donor subtree     */
/* until the child fits the stack).  Readings:                              */
/*  - stream tag 2, item = offspring index i, generation g; draw 0 picks    */
/*    the operation: u < pc crossover, < pc+ps subtree, < ..+ph hoist,      */
/*    < ..+pp point, else reproduction (running sums in float32);           */
/*  - crossover takes two tournaments (parent, then donor), every other     */
/*    operation one; offspring i's tournaments start at the prefix sum;     */
/*  - a random subtree is the one rooted at a uniformly drawn position;     */
/*  - crossover: parent subtree (draw 1) replaced by donor subtree (draw    */
/*    2); while the child's stack height exceeds 20 or its length max_len,  */
/*    the donor subtree becomes the one rooted at a uniformly drawn         */
/*    position strictly inside it (one draw each; it stops at a terminal);  */
/*  - subtree mutation: as crossover, the donor a program generated by the  */
/*    initialisation method on stream tag 3 (item i, generation g);         */
/*  - hoist: subtree (draw 1) replaced by the subtree rooted at a position  */
/*    drawn uniformly within it (draw 2, possibly its own root);            */
/*  - point: per node in prefix order one draw u; if u < p_replace the node */
/*    is replaced -- a function by one of the same arity (one draw over     */
/*    that arity's functions), a terminal by one of (features, constant)    */
/*    (one draw; a constant is allowed while the program's other constants  */
/*    number below max_consts, and takes one more draw for its value);     */
/*  - constants keep their values; slots are renumbered in prefix order.    */
/* ------------------------------------------------------------------------ */
static int draw_genetic_op(orc_rng *g, float pc, float ps, float ph, float pp)
{
    float t1 = pc;
    float t2 = t1 + ps;
    float t3 = t2 + ph;
    float t4 = t3 + pp;
    float u = word_unit(rng_word(g));
    if (u < t1) return 0;
    if (u < t2) return 1;
    if (u < t3) return 2;
    if (u < t4) return 3;
    return 4;
}

int orc_plan_generation(float pc, float ps, float ph, float pp, uint64_t seed, int32_t n_offspring,
                        uint64_t generation, int32_t *ops, int32_t *first_t, int32_t *n_t)
{
    int64_t t = 0;
    for (int32_t i = 0; i < n_offspring; ++i) {
        orc_rng g;
        rng_init(&g, seed, (uint32_t)i, (uint32_t)generation, 2u);
        ops[i] = draw_genetic_op(&g, pc, ps, ph, pp);
        first_t[i] = (int32_t)t;
        t += ops[i] == 0 ? 2 : 1;
    }
    *n_t = (int32_t)t;
    return 0;
}

/* a program as node words plus the value of each node's constant */
typedef struct { uint32_t *w; float *v; int64_t n; } orc_prog;

static orc_prog prog_alloc(int64_t n)
{
    orc_prog p;
    p.w = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    p.v = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    p.n = n;
    return p;
}
static void prog_free(orc_prog *p) { free(p->w); free(p->v); p->w = NULL; p->v = NULL; p->n = 0; }

/* end (one past) of the subtree rooted at s, by recursion on the arities */
static int64_t sub_end(const uint32_t *w, int64_t s)
{
    int ar = op_arity((int)(w[s] & 0xffu));
    int64_t e = s + 1;
    for (int a = 0; a < ar; ++a) e = sub_end(w, e);
    return e;
}

/* peak height of the right-to-left stack scan */
static int stack_peak(const uint32_t *w, int64_t n)
{
    int h = 0, m = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
        h += 1 - op_arity((int)(w[i] & 0xffu));
        if (h > m) m = h;
    }
    return m;
}

static orc_prog prog_from(const uint32_t *nodes, const int64_t *prog_off, const float *consts,
                          const int64_t *const_off, int32_t p)
{
    int64_t a = prog_off[p], n = prog_off[p + 1] - a;
    orc_prog r = prog_alloc(n);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t w = nodes[a + i];
        r.w[i] = w;
        r.v[i] = ((w & 0xffu) == O_CONST) ? consts[const_off[p] + (w >> 8)] : 0.0f;
    }
    return r;
}

/* parent with [s, e) replaced by donor [ds, de) */
static orc_prog replace_subtree(const orc_prog *par, int64_t s, int64_t e, const orc_prog *don,
                                int64_t ds, int64_t de)
{
    int64_t n = s + (de - ds) + (par->n - e), k = 0;
    orc_prog c = prog_alloc(n);
    for (int64_t i = 0; i < s; ++i, ++k) { c.w[k] = par->w[i]; c.v[k] = par->v[i]; }
    for (int64_t i = ds; i < de; ++i, ++k) { c.w[k] = don->w[i]; c.v[k] = don->v[i]; }
    for (int64_t i = e; i < par->n; ++i, ++k) { c.w[k] = par->w[i]; c.v[k] = par->v[i]; }
    return c;
}

static orc_prog hoisted_crossover(const orc_prog *par, const orc_prog *don, orc_rng *g, int32_t max_len)
{
    int64_t s = (int64_t)word_below(rng_word(g), (uint32_t)par->n);
    int64_t e = sub_end(par->w, s);
    int64_t ds = (int64_t)word_below(rng_word(g), (uint32_t)don->n);
    int64_t de = sub_end(don->w, ds);
    for (;;) {
        orc_prog c = replace_subtree(par, s, e, don, ds, de);
        if ((stack_peak(c.w, c.n) <= ORC_STACK && c.n <= max_len) || de - ds == 1) return c;
        prog_free(&c);
        ds = ds + 1 + (int64_t)word_below(rng_word(g), (uint32_t)(de - ds - 1));
        de = sub_end(don->w, ds);
    }
}

int orc_mutate(float pc, float ps, float ph, float pp, float p_replace, int32_t max_len, uint64_t seed,
               int32_t method, int32_t n_features, int32_t min_depth, int32_t max_depth,
               int32_t min_len, int32_t init_max_len, uint32_t fmask, float const_lo,
               float const_hi, int32_t max_consts,
               const uint32_t *nodes, const int64_t *prog_off, const float *consts,
               const int64_t *const_off, const int32_t *ops, const int32_t *first_t,
               const int32_t *winners, int32_t n_offspring, uint64_t generation,
               uint32_t *out_nodes, int64_t nodes_cap, int64_t *out_prog_off, float *out_consts,
               int64_t consts_cap, int64_t *out_const_off, int32_t *out_len,
               int64_t *total_nodes, int64_t *total_consts)
{
    (void)pc; (void)ps; (void)ph; (void)pp;
    orc_gen_cfg cfg;
    if (fill_cfg(&cfg, n_features, fmask, const_lo, const_hi, max_consts) != 0) return -1;
    int64_t nn = 0, ncs = 0;
    int overflow = 0;
    for (int32_t i = 0; i < n_offspring; ++i) {
        orc_rng g;
        rng_init(&g, seed, (uint32_t)i, (uint32_t)generation, 2u);
        (void)rng_word(&g);               /* the operation draw */
        orc_prog par = prog_from(nodes, prog_off, consts, const_off, winners[first_t[i]]);
        orc_prog child;
        if (ops[i] == 0) {
            orc_prog don = prog_from(nodes, prog_off, consts, const_off, winners[first_t[i] + 1]);
            child = hoisted_crossover(&par, &don, &g, max_len);
            prog_free(&don);
        } else if (ops[i] == 1) {
            /* the donor: a fresh program on the donor stream */
            orc_rng gd;
            rng_init(&gd, seed, (uint32_t)i, (uint32_t)generation, 3u);
            orc_buf b;
            b.nodes = NULL; b.consts = NULL;
            b.n = 0; b.nc = 0; b.cap = 0; b.ccap = 0; b.overflow = 0;
            orc_rng probe = gd;                              /* size pass */
            if (gen_one(&probe, &cfg, &b, method, min_depth, max_depth, min_len, init_max_len) != 0) return -1;
            int64_t dn = b.n, dc = b.nc;
            uint32_t *dw = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(dn > 0 ? dn : 1));
            float *dv = (float *)malloc(sizeof(float) * (size_t)(dc > 0 ? dc : 1));
            b.nodes = dw; b.cap = dn; b.consts = dv; b.ccap = dc; b.n = 0; b.nc = 0;
            gen_one(&gd, &cfg, &b, method, min_depth, max_depth, min_len, init_max_len);
            orc_prog don = prog_alloc(dn);
            for (int64_t k = 0; k < dn; ++k) {
                don.w[k] = dw[k];
                don.v[k] = ((dw[k] & 0xffu) == O_CONST) ? dv[dw[k] >> 8] : 0.0f;
            }
            free(dw); free(dv);
            child = hoisted_crossover(&par, &don, &g, max_len);
            prog_free(&don);
        } else if (ops[i] == 2) {
            int64_t s = (int64_t)word_below(rng_word(&g), (uint32_t)par.n);
            int64_t e = sub_end(par.w, s);
            int64_t s2 = s + (int64_t)word_below(rng_word(&g), (uint32_t)(e - s));
            int64_t e2 = sub_end(par.w, s2);
            child = replace_subtree(&par, s, e, &par, s2, e2);
        } else if (ops[i] == 3) {
            child = prog_alloc(par.n);
            int nconst = 0;
            for (int64_t k = 0; k < par.n; ++k) {
                child.w[k] = par.w[k]; child.v[k] = par.v[k];
                if ((par.w[k] & 0xffu) == O_CONST) nconst++;
            }
            for (int64_t k = 0; k < child.n; ++k) {
                float u = word_unit(rng_word(&g));
                if (!(u < p_replace)) continue;
                int op = (int)(child.w[k] & 0xffu);
                int ar = op_arity(op);
                if (ar == 1) {
                    if (cfg.n_un == 0) continue;
                    child.w[k] = (uint32_t)cfg.un[word_below(rng_word(&g), (uint32_t)cfg.n_un)];
                } else if (ar == 2) {
                    if (cfg.n_bin == 0) continue;
                    child.w[k] = (uint32_t)cfg.bin[word_below(rng_word(&g), (uint32_t)cfg.n_bin)];
                } else {
                    int others = nconst - (op == O_CONST ? 1 : 0);
                    int c_ok = cfg.consts_on && (cfg.max_consts <= 0 || others < cfg.max_consts);
                    int pick = (int)word_below(rng_word(&g), (uint32_t)(cfg.n_features + (c_ok ? 1 : 0)));
                    if (pick < cfg.n_features) {
                        child.w[k] = (uint32_t)O_VAR | ((uint32_t)pick << 8);
                        child.v[k] = 0.0f;
                        nconst = others;
                    } else {
                        child.w[k] = (uint32_t)O_CONST;
                        child.v[k] = draw_const(&g, &cfg);
                        nconst = others + 1;
                    }
                }
            }
        } else {
            child = prog_alloc(par.n);
            for (int64_t k = 0; k < par.n; ++k) { child.w[k] = par.w[k]; child.v[k] = par.v[k]; }
        }
        prog_free(&par);
        /* emit with constants renumbered in prefix order */
        if (out_prog_off) out_prog_off[i] = nn;
        if (out_const_off) out_const_off[i] = ncs;
        if (out_len) out_len[i] = (int32_t)child.n;
        int64_t slot = 0;
        for (int64_t k = 0; k < child.n; ++k) {
            uint32_t w = child.w[k];
            if ((w & 0xffu) == O_CONST) {
                if (out_consts && ncs + slot < consts_cap) out_consts[ncs + slot] = child.v[k];
                else overflow = 1;
                w = (uint32_t)O_CONST | ((uint32_t)slot << 8);
                slot++;
            }
            if (out_nodes && nn + k < nodes_cap) out_nodes[nn + k] = w; else overflow = 1;
        }
        nn += child.n;
        ncs += slot;
        prog_free(&child);
    }
    if (out_prog_off) out_prog_off[n_offspring] = nn;
    if (out_const_off) out_const_off[n_offspring] = ncs;
    *total_nodes = nn;
    *total_consts = ncs;
    return overflow ? -2 : 0;
}

