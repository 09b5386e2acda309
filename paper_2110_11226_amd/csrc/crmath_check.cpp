// crmath_check.cpp -- runs every float through gp_crmath.h's sin, cos and
// log (compiled for the host) and compares each result with the correctly
// rounded value decided from the C library: the double result of sin / cos /
// log (error below one double ulp) decides the rounding unless it lies within
// 8 double ulps of a float rounding boundary; then the extended-precision
// (long double) result decides, unless it too lies within 8 of its ulps of
// the boundary, and the input is printed as "undecided" for a
// higher-precision check.
//
// Two things are compared with that value: the plain rounding to float of
// the function's double result (before any exception-table lookup), whose
// misses are the exception-table entries whatever tables are compiled in,
// and the function itself, tables included, which must never miss.
//
// Output, one line per finding:
//   <op> <bits of x> <bits of the correctly rounded result>   an input the
//        double evaluation rounds wrongly (an exception-table entry)
//   unflagged <op> <bits>   such an input whose double result did not lie
//        near a rounding boundary: the error bound is wrong (never expected)
//   wrong <op> <bits> got <bits> want <bits>   the function (tables
//        included) returned another float: the tables are stale
//   undecided <op> <bits>   the reference could not decide
// and a summary per function: inputs, near a boundary, wrong, unflagged,
// undecided, exception entries.
//
// Build and run (host only):
//   g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -o crmath_check crmath_check.cpp
//   ./crmath_check [sin|cos|log|sign|all [stride]] > findings.txt
// ("sign" runs only the pass over negative inputs that sin and cos end with)
// Entries of the form "<op> <bits> <bits>" are the exception tables that
// gen_crmath_tables.py writes into gp_crmath_tables.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "gp_crmath.h"

namespace {

// Correctly rounded float of the exact value, decided from double v (error
// below 1 ulp) or long double w; returns false when neither can decide.
bool decide(double v, long double w, float* out) {
    float f = static_cast<float>(v);
    // distance of v from the nearest float rounding boundary in double ulps
    uint64_t b;
    std::memcpy(&b, &v, 8);
    const long long lo = static_cast<long long>(b & 0x1FFFFFFFull) - 0x10000000ll;
    if (lo > 8 || lo < -8) {
        *out = f;
        return true;
    }
    // the extended result: 64-bit significand, boundary at bit 39 below the top
    const float g = static_cast<float>(w);
    const long double gd = static_cast<long double>(g);
    // neighbouring floats of g and the two boundaries around it
    const float up = std::nextafter(g, INFINITY), dn = std::nextafter(g, -INFINITY);
    const long double mu = (gd + static_cast<long double>(up)) / 2, md = (gd + static_cast<long double>(dn)) / 2;
    const long double ulp = std::fabs(w) * 0x1p-63L;
    if (std::fabs(w - mu) <= 8 * ulp || std::fabs(w - md) <= 8 * ulp) return false;
    *out = g;
    return true;
}

struct Count {
    long long n = 0, flagged = 0, wrong = 0, unflagged = 0, undecided = 0, entries = 0;
};

long long g_stride = 1;   // every g_stride-th input (1: all of them)

template <typename Dev, typename Raw, typename Ref, typename RefL>
Count run(const char* name, uint32_t lo, uint32_t hi, Dev dev, Raw raw, Ref ref, RefL refl) {
    Count total;
#pragma omp parallel
    {
        Count c;
#pragma omp for schedule(dynamic, 1 << 16)
        for (long long ub = lo; ub <= static_cast<long long>(hi); ub += g_stride) {
            float x;
            const uint32_t u = static_cast<uint32_t>(ub);
            std::memcpy(&x, &u, 4);
            ++c.n;
            const float got = dev(x);
            const double y = raw(x);
            const float plain = static_cast<float>(y);
            const bool fl = gp::crm::near_boundary(y);
            if (fl) ++c.flagged;
            float want;
            if (!decide(ref(static_cast<double>(x)), refl(static_cast<long double>(x)), &want)) {
                ++c.undecided;
#pragma omp critical
                std::printf("undecided %s 0x%08x\n", name, u);
                continue;
            }
            uint32_t gb, pb, wb;
            std::memcpy(&gb, &got, 4);
            std::memcpy(&pb, &plain, 4);
            std::memcpy(&wb, &want, 4);
            if (pb != wb) {
                ++c.entries;
                if (!fl) ++c.unflagged;
#pragma omp critical
                {
                    if (fl)
                        std::printf("%s 0x%08x 0x%08x\n", name, u, wb);
                    else
                        std::printf("unflagged %s 0x%08x got 0x%08x want 0x%08x\n", name, u, pb, wb);
                }
            }
            if (gb != wb) {
                ++c.wrong;
#pragma omp critical
                std::printf("wrong %s 0x%08x got 0x%08x want 0x%08x\n", name, u, gb, wb);
            }
        }
#pragma omp critical
        {
            total.n += c.n;
            total.flagged += c.flagged;
            total.wrong += c.wrong;
            total.unflagged += c.unflagged;
            total.undecided += c.undecided;
            total.entries += c.entries;
        }
    }
    std::fprintf(stderr, "%s: %lld inputs, %lld near a boundary, %lld exception entries (%lld unflagged), "
                 "%lld wrong with the tables, %lld undecided\n", name, total.n, total.flagged, total.entries,
                 total.unflagged, total.wrong, total.undecided);
    std::printf("summary %s %lld %lld %lld %lld %lld %lld\n", name, total.n, total.flagged, total.wrong,
                total.unflagged, total.undecided, total.entries);
    return total;
}

// the double result each function rounds to float (before its exception
// tables)
double raw_sincos(float x, bool is_cos) {
    const float ax = std::fabs(x);
    uint32_t ub;
    std::memcpy(&ub, &ax, 4);
    const gp::crm::SinCosK K = gp::crm::sincos_k(is_cos);
    return ax < 0x1p+20f ? gp::crm::sincos_small(ax, gp::crm::kSinCosTab, K)
                         : gp::crm::sincos_large(ub, is_cos, gp::crm::kSinCosTab, K);
}
double raw_sin(float x) { return raw_sincos(x, false); }
double raw_cos(float x) { return raw_sincos(x, true); }
double raw_log(float x) { return gp::crm::log_double(x, gp::crm::kLogTab, gp::crm::log_k()); }

}  // namespace

int main(int argc, char** argv) {
    const char* which = argc > 1 ? argv[1] : "all";
    if (argc > 2) g_stride = std::max(1LL, std::atoll(argv[2]));
    // an optional range of input bits [lo, hi] replaces every function's own
    // (and skips the sign pass)
    const bool ranged = argc > 4;
    const uint32_t rlo = ranged ? static_cast<uint32_t>(std::strtoul(argv[3], nullptr, 0)) : 0u;
    const uint32_t rhi = ranged ? static_cast<uint32_t>(std::strtoul(argv[4], nullptr, 0)) : 0u;
    uint32_t fin = 0x7F7FFFFFu;   // largest finite float
    float t = 0.001f;
    uint32_t logs;
    std::memcpy(&logs, &t, 4);
    uint32_t slo = 0u;
    if (ranged) {
        slo = rlo;
        logs = rlo - 1;   // (log starts at logs + 1)
        fin = rhi;
    }
    if (!std::strcmp(which, "all") || !std::strcmp(which, "sin"))
        run("sin", slo, fin, [](float x) { return gp::crm::sin_cr(x, gp::crm::kSinCosTab, gp::crm::sincos_k(false)); }, raw_sin,
            [](double x) { return std::sin(x); }, [](long double x) { return sinl(x); });
    if (!std::strcmp(which, "all") || !std::strcmp(which, "cos"))
        run("cos", slo, fin, [](float x) { return gp::crm::cos_cr(x, gp::crm::kSinCosTab, gp::crm::sincos_k(true)); }, raw_cos,
            [](double x) { return std::cos(x); }, [](long double x) { return cosl(x); });
    if (!ranged && (!std::strcmp(which, "all") || !std::strcmp(which, "sin") || !std::strcmp(which, "cos") ||
                    !std::strcmp(which, "sign"))) {
        // negative inputs: sin(-x) = -sin x and cos(-x) = cos x bit for bit
        // (both zeros, infinities and NaN included), on every g_stride-th float
        long long bad = 0, n = 0;
        const gp::crm::SinCosK KS = gp::crm::sincos_k(false), KC = gp::crm::sincos_k(true);
#pragma omp parallel for reduction(+ : bad, n) schedule(dynamic, 1 << 16)
        for (long long ub = 0; ub <= 0x7FFFFFFFll; ub += g_stride) {
            float x, nx;
            const uint32_t u = static_cast<uint32_t>(ub), nu = u | 0x80000000u;
            std::memcpy(&x, &u, 4);
            std::memcpy(&nx, &nu, 4);
            const float sp = gp::crm::sin_cr(x, gp::crm::kSinCosTab, KS), sn = gp::crm::sin_cr(nx, gp::crm::kSinCosTab, KS);
            const float cp = gp::crm::cos_cr(x, gp::crm::kSinCosTab, KC), cn = gp::crm::cos_cr(nx, gp::crm::kSinCosTab, KC);
            const float msp = -sp;
            uint32_t a, b, c, d;
            std::memcpy(&a, &msp, 4);
            std::memcpy(&b, &sn, 4);
            std::memcpy(&c, &cp, 4);
            std::memcpy(&d, &cn, 4);
            const bool nan = std::isnan(sp) && std::isnan(sn) && std::isnan(cp) && std::isnan(cn);
            ++n;
            if (!nan && (a != b || c != d)) {
                ++bad;
#pragma omp critical
                std::printf("sign 0x%08x sin %08x/%08x cos %08x/%08x\n", nu, b, a, d, c);
            }
        }
        std::printf("summary sign %lld 0 %lld %lld 0 0\n", n, bad, bad);
    }
    if (!std::strcmp(which, "all") || !std::strcmp(which, "log"))
        run("log", logs + 1, fin, [](float x) { return gp::crm::log_cr(x, gp::crm::kLogTab, gp::crm::log_k()); }, raw_log,
            [](double x) { return std::log(x); }, [](long double x) { return logl(x); });
    return 0;
}
