// Host driver for the secondary-uncertainty draw's logarithm, cosine of
// 2 pi u and exponential (su_math.h): evaluates them on the host over the
// arguments the draw gives and prints the largest error against the C
// library in units in the last place (and the cosine's absolute error in
// units of 2^-53).  Built by tests/test_su_math_cpu.py.
#include "su_math.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

static double ulps(double got, double ref) {
    if (got == ref) return 0.0;
    if (!std::isfinite(got) || !std::isfinite(ref)) return 1e300;
    const double a = std::fabs(ref);
    const double u = std::nextafter(a, INFINITY) - a;
    return std::fabs(got - ref) / u;
}

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014)
static uint64_t next(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main(int argc, char **argv) {
    const long n = argc > 1 ? std::atol(argv[1]) : 1000000;
    uint64_t s = 1308257203ull;
    double wl = 0, wc = 0, wca = 0, we = 0, wez = 0;
    auto cosref = [](double u) { return std::cos(ara::sumath::kTwoPi * u); };
    auto check_u = [&](double u) {
        wl = std::fmax(wl, ulps(ara::su_log(u), std::log(u)));
        const double c = ara::su_cos_2pi(u), r = cosref(u);
        wca = std::fmax(wca, std::fabs(c - r) * 0x1p53);
        if (std::fabs(r) >= 0x1p-10) wc = std::fmax(wc, ulps(c, r));
    };
    for (long i = 0; i < n; ++i) {
        // the draw's uniforms: (52 random bits + 1/2) 2^-52
        check_u((static_cast<double>(next(s) >> 12) + 0.5) * 0x1p-52);
        // exponents of the draws: m + s z lies well inside [-60, 60]
        const double y = -60.0 + 120.0 * (static_cast<double>(next(s) >> 11) * 0x1p-53);
        we = std::fmax(we, ulps(ara::su_exp(y), std::exp(y)));
    }
    // ends of the uniforms' range, quadrant boundaries and powers of two
    const double us[] = {0x1p-53, 0x1p-52, 0x1.8p-52, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 1.0 - 0x1p-53, 1.0};
    for (double u : us) check_u(u);
    for (int e = -52; e < 0; ++e) check_u(std::ldexp(1.0, e));
    // the exponential's ends: results at and past the binary64 range
    const double ys[] = {0.0, -0.0, 1.0, -1.0, 700.0, 709.78, 709.79, 720.0, 1e300, -700.0, -708.0, -745.0, -746.0,
                         -760.0, -1e300};
    for (double y : ys) {
        const double g = ara::su_exp(y), r = std::exp(y);
        const double err = (r == 0.0 || std::isinf(r)) ? (g == r ? 0.0 : 1e300)
                         : (r < 0x1p-1022 ? std::fabs(g - r) / 0x1p-1074 : ulps(g, r));
        wez = std::fmax(wez, err);
    }
    std::printf("log %.3f\ncos %.3f\ncos_abs %.3f\nexp %.3f\nexp_edges %.3f\n", wl, wc, wca, we, wez);
    return 0;
}
