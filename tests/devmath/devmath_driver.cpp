// Host driver for tests/test_devmath.py: evaluates the trace kernels' compact
// elementary functions (paper_2605_05635_amd/csrc/rt_math.h, compiled for the
// host) on the doubles read from stdin and writes the results to stdout.
//   usage: devmath_driver <function>   (sincos | exp | expm1 | expm1_near | log1p | log1p_fast | rpow_tenth, and the
//          binary32 versions sincosf | expf | expm1f | log1pf of the arguments rounded
//          to binary32; cnfw_terms reads (R, lambda_c) pairs and writes 1/R,
//          1/(R + lambda_c) and log(1 + R/lambda_c))
#include <cstdio>
#include <cstring>
#include <vector>

#include "rt_device.h"
#include "rt_math.h"

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    std::vector<double> x;
    double v;
    while (std::fread(&v, sizeof v, 1, stdin) == 1) x.push_back(v);
    std::vector<double> out;
    if (!std::strcmp(argv[1], "cnfw_terms")) {
        for (size_t i = 0; i + 1 < x.size(); i += 2) {
            const rt::CnfwTerms t = rt::cnfw_terms(x[i], x[i + 1], 1.0 / x[i + 1]);
            out.push_back(t.iR);
            out.push_back(t.iRl);
            out.push_back(t.lg);
        }
        std::fwrite(out.data(), sizeof(double), out.size(), stdout);
        return 0;
    }
    for (double a : x) {
        if (!std::strcmp(argv[1], "sincos")) {
            double s, c;
            rt::dm::sincos(a, &s, &c);
            out.push_back(s);
            out.push_back(c);
        } else if (!std::strcmp(argv[1], "exp")) {
            out.push_back(rt::dm::exp(a));
        } else if (!std::strcmp(argv[1], "expm1")) {
            out.push_back(rt::dm::expm1(a));
        } else if (!std::strcmp(argv[1], "expm1_near")) {
            out.push_back(rt::dm::expm1_near(a));
        } else if (!std::strcmp(argv[1], "log1p")) {
            out.push_back(rt::dm::log1p(a));
        } else if (!std::strcmp(argv[1], "log1p_fast")) {
            out.push_back(rt::dm::log1p_fast(a));
        } else if (!std::strcmp(argv[1], "rpow_tenth")) {
            out.push_back(rt::dm::rpow_tenth(a));
        } else if (!std::strcmp(argv[1], "sincosf")) {
            float s, c;
            rt::dm::sincos(static_cast<float>(a), &s, &c);
            out.push_back(s);
            out.push_back(c);
        } else if (!std::strcmp(argv[1], "expf")) {
            out.push_back(rt::dm::exp(static_cast<float>(a)));
        } else if (!std::strcmp(argv[1], "expm1f")) {
            out.push_back(rt::dm::expm1(static_cast<float>(a)));
        } else if (!std::strcmp(argv[1], "log1pf")) {
            out.push_back(rt::dm::log1p(static_cast<float>(a)));
        } else {
            return 3;
        }
    }
    std::fwrite(out.data(), sizeof(double), out.size(), stdout);
    return 0;
}
