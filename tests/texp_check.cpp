// CPU check of the table-driven double exp of pins_texp.h against the host
// libm exp: largest error in ulps of the reference over random and edge
// arguments in [-746, 710] (subnormal results included), and the special
// cases (underflow to 0, overflow to inf, NaN).  Prints one line
// "max_ulp <e> worst_x <x> n <count> special_ok <0|1>"; test infrastructure.
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "pins_texp.h"

static double ulp_of(double y) {
    if (y == 0.0) return std::nextafter(0.0, 1.0);
    const double a = std::fabs(y);
    return std::nextafter(a, INFINITY) - a;
}

int main(int argc, char** argv) {
    const long n = argc > 1 ? std::atol(argv[1]) : 20000000L;
    double T[64];
    for (int j = 0; j < 64; ++j) T[j] = pins::texp_table_entry(j);
    std::mt19937_64 g(250203749);
    std::uniform_real_distribution<double> U(-746.0, 710.0), Usub(-745.2, -708.0), Usmall(-1.0, 1.0);
    double worst = 0.0, wx = 0.0;
    long count = 0;
    auto check = [&](double x) {
        const double ref = std::exp(x), got = pins::texp_eval(x, T);
        if (std::isinf(ref) || std::isinf(got)) {
            if (!(std::isinf(ref) && std::isinf(got))) { worst = INFINITY; wx = x; }
        } else {
            const double e = std::fabs(got - ref) / ulp_of(ref);
            if (e > worst) { worst = e; wx = x; }
        }
        ++count;
    };
    for (long i = 0; i < n; ++i) check(U(g));
    for (long i = 0; i < n / 8; ++i) check(Usub(g));
    for (long i = 0; i < n / 8; ++i) check(Usmall(g));
    // edges: every multiple of ln2/64 near 0 and the range ends, and their neighbours
    const double h = 0.6931471805599453 / 64.0;
    for (int k = -64 * 1100; k <= 64 * 1030; ++k) {
        const double x = k * h;
        if (x < -746.0 || x > 710.0) continue;
        check(x);
        check(std::nextafter(x, -INFINITY));
        check(std::nextafter(x, INFINITY));
    }
    const double edges[] = {0.0, -0.0, 1e-300, -1e-300, 709.78, 709.7827128933840, 709.79, -708.39, -745.13,
                            -745.1332191019412, -745.14, -746.0, 710.0};
    for (double x : edges) check(x);
    bool special = pins::texp_eval(-746.5, T) == 0.0 && pins::texp_eval(-1e6, T) == 0.0 &&
                   pins::texp_eval(-INFINITY, T) == 0.0 && std::isinf(pins::texp_eval(710.5, T)) &&
                   std::isinf(pins::texp_eval(INFINITY, T)) && std::isinf(pins::texp_eval(1e300, T)) &&
                   std::isnan(pins::texp_eval(NAN, T)) && pins::texp_eval(0.0, T) == 1.0;
    // the non-positive form: bitwise the general one for x <= 0 (and 0 for -inf)
    long nonpos_diff = 0;
    for (long i = 0; i < n / 4; ++i) {
        const double x = -std::fabs(U(g));
        if (pins::texp_eval_nonpos(x, T) != pins::texp_eval(x, T)) ++nonpos_diff;
    }
    for (double x : {0.0, -0.0, -746.0, -745.5, -1e6, -(double)INFINITY})
        if (pins::texp_eval_nonpos(x, T) != pins::texp_eval(x, T)) ++nonpos_diff;
    std::printf("max_ulp %.6g worst_x %.17g n %ld special_ok %d nonpos_diff %ld\n", worst, wx, count,
                special ? 1 : 0, nonpos_diff);
    return 0;
}
