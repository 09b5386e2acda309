// gp_crmath.h -- correctly rounded float32 sin, cos and log for the
// evaluation kernels.
//
// The function set of Sec. III-D1 names sin, cos and log but no library; a
// float32 evaluation that rounds each function's exact value once, to
// nearest (ties to even), as IEEE arithmetic does for +, -, *, / and sqrt,
// makes a program's float32 value independent of which library computed it.
// With these three, every function of the benchmark set {add, sub, mul,
// protected div, neg, protected log, protected sqrt, sin, cos} is correctly
// rounded, so a program's output is one fixed float32 number per row.
//
// Method (each function): the float argument is widened to double (exact),
// the function is evaluated in double with a relative error below 2^-50,
// and the result is rounded to float.  That rounding is the correctly
// rounded one unless the double result lies within the error bound of a
// float rounding boundary (the midpoint of two neighbouring floats); there,
// and only there, an exception table holds the inputs whose double result
// falls on the wrong side (found by running every float through these
// functions against an independent reference, crmath_check.cpp).
//
//   sin, cos: x = k (pi/64) + r, |r| <= pi/128: for |x| < 2^20 by a
//     three-part Cody-Waite reduction whose first two products are exact;
//     beyond, by Payne-Hanek on |x|: the 24-bit mantissa times a 160-bit
//     window of the binary digits of 2/pi, in 32-bit integer limbs.  Then
//     sin x = S cos r + C sin r with S, C the sine and cosine of
//     (k mod 128) pi/64 from a table (cos x takes k + 32), sin r and cos r by
//     short Taylor polynomials.
//   log: a = 2^e m, m in [1, 2); c = 1/(bucket centre of m) from a 128-entry
//     table (c has 24 bits, so m c - 1 is exact); log a = E ln 2 - log c' +
//     log1p(m c - 1) with log1p to r^7 (|m c - 1| <= 2^-7), the table's
//     -log c' and ln 2 each rounded to double.
// The code is host- and device-compilable so that the exhaustive checker can
// run the very same functions on the CPU.  The tables are taken by pointer
// (the evaluation kernels stage them in LDS) and the double constants as a
// struct (sincos_k, log_k: built once per instruction, shared by the rows a
// lane evaluates).
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define GP_CRF __host__ __device__ __forceinline__
#define GP_CRTAB __device__ static constexpr
#else
#include <cmath>
#define GP_CRF inline
#define GP_CRTAB static constexpr
#endif

#include "gp_crmath_tables.h"

namespace gp {
namespace crm {

// A constant handed to a double FMA through a scalar register pair: it is
// then an operand of v_fma_f64 itself, instead of a vector register pair
// the compiler would fill with two moves per use or keep occupied for the
// whole kernel.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ double kreg(double c) {
    asm volatile("" : "+s"(c));
    return c;
}
// The same constant in a vector register pair: the operand of an FMA whose
// other two operands already include a scalar one (one scalar operand per
// vector instruction), set once and shared by the rows of a lane.
__device__ __forceinline__ double kvreg(double c) {
    double v;
    asm volatile("v_mov_b64 %0, %1" : "=v"(v) : "s"(c));
    return v;
}
#else
inline double kreg(double c) { return c; }
inline double kvreg(double c) { return c; }
#endif

GP_CRF uint64_t dbits(double v) {
    uint64_t u;
    __builtin_memcpy(&u, &v, sizeof u);
    return u;
}
GP_CRF uint32_t fbits(float v) {
    uint32_t u;
    __builtin_memcpy(&u, &v, sizeof u);
    return u;
}
GP_CRF float bitsf(uint32_t u) {
    float v;
    __builtin_memcpy(&v, &u, sizeof v);
    return v;
}

// Rounding the double y to float can differ from rounding the exact value
// only if y lies within its error bound of a float rounding boundary: the
// 29 bits below float precision within kHardUlps double ulps of one half.
// (The error bound 2^-50 |y| is at most 2^3 double ulps of y; 16 doubles it.)
constexpr uint32_t kHardUlps = 16;
GP_CRF bool near_boundary(double y) {
    const uint32_t lo = static_cast<uint32_t>(dbits(y)) & 0x1FFFFFFFu;
    return lo - (0x10000000u - kHardUlps) <= 2u * kHardUlps;
}

// The correctly rounded result of an input the exception table lists, else
// the rounding f of the double result.
template <int N>
GP_CRF float exception(const uint32_t (&tab)[N][2], int n, uint32_t key, float f) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("");   // keeps the search behind its (rarely taken) branch
#endif
    for (int i = 0; i < n; ++i)
        if (tab[i][0] == key) return bitsf(tab[i][1]);
    return f;
}

// ---- sin, cos ----
// |x| = k (pi/64) + r, |r| <= pi/128; with j = k mod 128 (plus 32 for cos,
// cos x = sin(x + pi/2)), sin x = S_j cos r + C_j sin r for S_j, C_j the
// sine and cosine of j pi/64 from a table, cos r - 1 and sin r by their
// Taylor polynomials through r^6 and r^7 (truncation below 2^-57 relative).
constexpr double kInvPi64 = 0x1.45f306dc9c883p+4;   // 64/pi
// pi/64 = kPi64a + kPi64b + kPi64c + O(2^-119): a and b carry at most 28
// bits, so k * a and k * b are exact for k < 2^25 (|x| < 2^20)
constexpr double kPi64a = 0x1.921fb54000000p-5;
constexpr double kPi64b = 0x1.10b4610000000p-35;
constexpr double kPi64c = 0x1.a62633145c06ep-63;
constexpr double kPi64 = 0x1.921fb54442d18p-5;
// (-1)^n / (2n+1)! and (-1)^n / (2n)!
constexpr double kS3 = -0x1.5555555555555p-3, kS5 = 0x1.1111111111111p-7, kS7 = -0x1.a01a01a01a01ap-13;
constexpr double kC4 = 0x1.5555555555555p-5, kC6 = -0x1.6c16c16c16c17p-10;

// 1.5 * 2^52: x + kRound is x rounded to an integer, held in the low bits of
// the double's significand (|x| < 2^51); cos adds its quarter turn, 32
// table steps, in the same operation
constexpr double kRound = 0x1.8p+52;
constexpr double kRoundCos = 0x1.8p+52 + 32.0;

// The double constants of sin (is_cos false) or cos as operands.  The
// evaluation kernels build this once per instruction and share it among the
// rows a lane holds.
struct SinCosK {
    double inv, rnd, pa, pb, pc, s3, s5, s7, c4, c6;
};
GP_CRF SinCosK sincos_k(bool is_cos) {
    return SinCosK{kreg(kInvPi64), kreg(is_cos ? kRoundCos : kRound), kreg(kPi64a), kreg(kPi64b),
                   kreg(kPi64c),   kreg(kS3), kvreg(kS5), kreg(kS7), kvreg(kC4), kreg(kC6)};
}

// sin(j pi/64 + r) for |r| <= pi/128 (slightly more after rounding of k)
GP_CRF double sin_from_table(const SinCosEntry& e, double r, const SinCosK& K) {
    const double r2 = r * r;
    const double sp = fma(fma(K.s7, r2, K.s5), r2, K.s3);
    const double cp = fma(fma(K.c6, r2, K.c4), r2, -0.5);
    const double cm1 = r2 * cp;                  // cos r - 1
    const double sr = fma(r * r2, sp, r);        // sin r
    return fma(e.s, cm1, fma(e.c, sr, e.s));
}

// |x| <= 2^20: k and r by a three-part Cody-Waite reduction.  k is the
// integer nearest x * 64/pi (from the exact product: a tie or a
// neighbouring integer only moves r within the polynomials' range), and
// the low word of x * 64/pi + K.rnd is k (k + 32 for cos) modulo 2^32, so
// that a negative k indexes the table as k mod 128 does.  Every step is odd
// in x (k, r and the table's sines change sign, its cosines do not), so
// sin(-x) = -sin x and cos(-x) = cos x hold bit for bit, zeros aside (see
// sincos_common).
GP_CRF double sincos_small(double x, const SinCosEntry* tab, const SinCosK& K) {
    const double kr = fma(x, K.inv, K.rnd);
    const double k = kr - K.rnd;
    double r = fma(-k, K.pa, x);
    r = fma(-k, K.pb, r);
    r = fma(-k, K.pc, r);
    // byte offset of entry (k or k + 32) mod 128
    const uint32_t off = (static_cast<uint32_t>(dbits(kr)) << 4) & 0x7F0u;
    return sin_from_table(*reinterpret_cast<const SinCosEntry*>(reinterpret_cast<const char*>(tab) + off), r, K);
}

// The binary digits of 2/pi in 32-bit words, after one word of zeros (the
// word index of digit p >= 1, weight 2^-p, is (p + 31) / 32).
GP_CRTAB uint32_t kTwoOverPi[13] = {0u,          0xa2f9836eu, 0x4e441529u, 0xfc2757d1u, 0xf534ddc0u,
                                   0xdb629599u, 0x3c439041u, 0xfe5163abu, 0xdebbc561u, 0xb7246e3au,
                                   0x424dd2e0u, 0x06492eeau, 0x09d1921cu};

// Payne-Hanek for finite |x| = M 2^E >= 2^20 (ub: the float bits of |x|).
// Digits of 2/pi of weight 2^(E-p) >= 4 multiply the integer M into
// multiples of 4 and are dropped: the window is digits p = E-1 .. E+158 (160
// bits), so Z = M * window * 2^-158 = |x| 2/pi mod 4 carries 158 fraction
// bits and an error below 2^-134.  32 Z = |x| 64/pi mod 128: k is its
// nearest integer (bits 153 up, after adding 2^152) and r = (32 Z - k) pi/64.
GP_CRF double sincos_large(uint32_t ub, bool is_cos, const SinCosEntry* tab, const SinCosK& K) {
    const uint32_t M = (ub & 0x7FFFFFu) | 0x800000u;
    const int E = static_cast<int>(ub >> 23) - 150;
    const int p0 = E - 1;
    const int k0 = (p0 + 31) >> 5;
    const int s = (p0 + 31) & 31;
    uint32_t z[5];
    uint64_t c = 0;
    for (int j = 4; j >= 0; --j) {
        const uint32_t w = s ? (kTwoOverPi[k0 + j] << s) | (kTwoOverPi[k0 + j + 1] >> (32 - s))
                             : kTwoOverPi[k0 + j];
        const uint64_t t = static_cast<uint64_t>(M) * w + c;
        z[j] = static_cast<uint32_t>(t);
        c = t >> 32;
    }
    // bit 152 of Z is bit 24 of z[0]; k = bits 153..159
    z[0] += 0x1000000u;
    const int k = static_cast<int>(z[0] >> 25);
    const int j = (k + (is_cos ? 32 : 0)) & 127;
    // D = (bits 0..152) - 2^152: signed, 153 fraction bits of 32 Z
    const int64_t top = static_cast<int64_t>(z[0] & 0x1FFFFFFu) - 0x1000000ll;
    const bool dneg = top < 0;
    uint32_t d[5] = {static_cast<uint32_t>(top), z[1], z[2], z[3], z[4]};
    if (dneg) {   // |D|: two's complement negation across the limbs
        uint64_t b = 1;
        for (int i = 4; i >= 0; --i) {
            const uint64_t t = static_cast<uint64_t>(~d[i]) + b;
            d[i] = static_cast<uint32_t>(t);
            b = t >> 32;
        }
    }
    // normalise |D| to 64 significant bits
    int j0 = 0;
    while (j0 < 2 && d[j0] == 0u) ++j0;
    const int l = __builtin_clz(d[j0] | 1u);   // (d[j0] != 0 for every float input)
    uint64_t hi = (static_cast<uint64_t>(d[j0]) << 32) | d[j0 + 1];
    if (l) hi = (hi << l) | (d[j0 + 2] >> (32 - l));
    double D = ldexp(static_cast<double>(hi), 160 - 64 - 153 - 32 * j0 - l);
    if (dneg) D = -D;
    return sin_from_table(tab[j], D * kPi64, K);
}

// Exception-table entries [B, E) (sorted by key) applied to f without a
// branch; an entry's result is negated where neg holds
template <int N>
GP_CRF float exceptions_select(const uint32_t (&tab)[N][2], int b, int e, uint32_t key, float f, bool neg) {
    for (int i = b; i < e; ++i) f = key == tab[i][0] ? (neg ? -bitsf(tab[i][1]) : bitsf(tab[i][1])) : f;
    return f;
}

// Correctly rounded sin (is_cos false) or cos of a float, in two parts so
// that a lane holding several rows can test them all before one branch:
// sincos_common is the result for |x| < 2^20, without a branch (exception
// entries below 2^20 are matched by selects); an input for which
// sincos_rare_input holds (|x| >= 2^20, inf, NaN) takes sincos_rare's
// result instead: Payne-Hanek reduction, or NaN.  Tiny arguments need no
// case of their own: for |x| < 2^-12 the double result lies within
// x^2 / 6 < 2^-26.6 (relative) of x, or x^2 / 2 < 2^-25 of 1, so it rounds
// to x (sin) or 1 (cos), as the exact value does.
GP_CRF float sincos_common(float x, bool is_cos, const SinCosEntry* tab, const SinCosK& K) {
    // (an input sincos_rare_input flags gets a meaningless value here, read
    // from within the table since its offset is masked, and replaced by
    // sincos_rare's)
    const double y = sincos_small(static_cast<double>(x), tab, K);
    float f = static_cast<float>(y);
    // (the entries list |x|; sin's result takes the sign of x)
    const uint32_t ub = fbits(x) & 0x7FFFFFFFu;
    if (is_cos) return exceptions_select(kCosExc, 0, kCosExcSmallN, ub, f, false);
    f = exceptions_select(kSinExc, 0, kSinExcSmallN, ub, f, (fbits(x) >> 31) != 0u);
    // sin(-0) = -0: the polynomial's additions of +0 give +0 there
    return x == 0.0f ? x : f;
}

GP_CRF bool sincos_rare_input(float x) { return !(fabsf(x) < 0x1p+20f); }   // (NaN included)

GP_CRF float sincos_rare(float x, bool is_cos, const SinCosEntry* tab, const SinCosK& K) {
    const uint32_t ub = fbits(x) & 0x7FFFFFFFu;
    float f;
    if (ub < 0x7F800000u) {
        const double yl = sincos_large(ub, is_cos, tab, K);
        f = static_cast<float>(yl);
        if (near_boundary(yl))
            f = is_cos ? exception(kCosExc, kCosExcN, ub, f) : exception(kSinExc, kSinExcN, ub, f);
    } else {
        f = x - x;   // NaN
    }
    return (!is_cos && (fbits(x) >> 31)) ? -f : f;
}

GP_CRF float sincos_cr(float x, bool is_cos, const SinCosEntry* tab, const SinCosK& K) {
    float f = sincos_common(x, is_cos, tab, K);
    if (sincos_rare_input(x)) f = sincos_rare(x, is_cos, tab, K);
    return f;
}

GP_CRF float sin_cr(float x, const SinCosEntry* tab, const SinCosK& K) { return sincos_cr(x, false, tab, K); }
GP_CRF float cos_cr(float x, const SinCosEntry* tab, const SinCosK& K) { return sincos_cr(x, true, tab, K); }

// ---- log ----
// ln 2 rounded to double: E ln 2 is then off by |E| 2^-55.3 at most, which
// is below 2^-53.8 of the result for every E != 0 (|log a| >= |E| ln 2 -
// ln(2)/2 there)
constexpr double kLn2 = 0x1.62e42fefa39efp-1;
// (-1)^(k+1) / k, k = 3..7 (log1p to r^7: |r| <= 2^-8, 2^-7 in the first
// bucket, whose c = 1; truncation below 2^-52 relative)
constexpr double kL3 = 0x1.5555555555555p-2, kL4 = -0x1.0000000000000p-2, kL5 = 0x1.999999999999ap-3,
                 kL6 = -0x1.5555555555555p-3, kL7 = 0x1.2492492492492p-3;

struct LogK {
    double l3, l4, l5, l6, l7, ln2;
};
GP_CRF LogK log_k() {
    return LogK{kreg(kL3), kreg(kL4), kreg(kL5), kvreg(kL6), kreg(kL7), kreg(kLn2)};
}

// log a for a normal positive finite float, in double: E ln 2 + L + log1p(r)
// with r = m c - 1 exact (24-bit m times the 24-bit c).  The table's L
// carries its double rounding, below 2^-53 |L|.  Where E = 0 and L != 0,
// |r| <= 0.34 |L|, so the result is at least 0.66 |L| and that rounding is
// below 2^-52.4 of it; with the rounding of log1p and of the final addition
// the relative error stays below 2^-51 (E ln 2 + L is exact when E = 0).
GP_CRF double log_double(float a, const LogEntry* tab, const LogK& K) {
    const uint32_t u = fbits(a);
    const int i = static_cast<int>((u >> 16) & 0x7Fu);
    const int E = static_cast<int>(u >> 23) - 127 + (i >= 53 ? 1 : 0);
    const double m = static_cast<double>(bitsf((u & 0x7FFFFFu) | 0x3F800000u));
    const LogEntry& t = tab[i];
    const double r = fma(m, t.c, -1.0);   // exact
    double p = fma(K.l7, r, K.l6);
    p = fma(p, r, K.l5);
    p = fma(p, r, K.l4);
    p = fma(p, r, K.l3);
    p = fma(p, r, -0.5);
    const double l1p = fma(r * r, p, r);
    return fma(static_cast<double>(E), K.ln2, t.hi) + l1p;
}

// Correctly rounded log of a float a > 0 that is normal, +inf or NaN (the
// protected log only takes |a| > 0.001).
GP_CRF float log_cr(float a, const LogEntry* tab, const LogK& K) {
    const double y = log_double(a, tab, K);   // (finite for +inf and NaN; replaced below)
    float f = static_cast<float>(y);
    if (near_boundary(y)) f = exception(kLogExc, kLogExcN, fbits(a), f);
    return a <= 0x1.fffffep+127f ? f : a;     // +inf (and NaN) unchanged
}

}  // namespace crm
}  // namespace gp
