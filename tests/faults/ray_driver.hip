// Host driver for tests/test_ray_faults.py: runs the trace kernels' per-ray
// step loop (paper_2605_05635_amd/csrc/rt_ray.h, compiled for the host from
// the same source) from a given initial state, with a fault forced from the
// host: attempts numbered first..last (1-based) see a spin of NaN, so every
// stage of those attempts is not finite, as a fault in the arithmetic would
// make it.
//
//   ray_driver  row = metric chi m0 m1 m2 E L R th pR pth rtol r_stop r_esc
//                     max_attempts first last
//     out: status, attempts, ncross, R at the end
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rt_ray.h"

using namespace rt;

namespace {

template <int M>
void ray_case(const double* a, std::vector<double>& out) {
    ImageConst c;
    std::memset(&c, 0, sizeof c);
    c.metric = M;
    c.chi = a[1];
    c.chi2 = a[1] * a[1];
    if (M == EINASTO) c.inv_lam = a[2];
    if (M == CNFW) {
        c.lam_c = a[2];
        c.inv_lam_c = a[3];
        c.eta_lc = a[4];
    }
    c.rtol = c.atol = a[11];
    c.r_stop = a[12];
    c.r_esc = a[13];
    c.max_attempts = static_cast<int32_t>(a[14]);
    c.n_pix = 1;
    const int first = static_cast<int>(a[15]), last = static_cast<int>(a[16]);
    const ray::Hot good = ray::hot_of(c);
    ray::Hot bad = good;
    bad.chi = std::nan("");
    ray::Ray r;
    std::memset(&r, 0, sizeof r);
    ray::set_constants(good.chi, a[5], a[6], r);
    r.y[1] = a[7];
    r.y[2] = a[8];
    r.y[4] = a[9];
    r.y[5] = a[10];
    ray::rhs<M>(good, r.E, r.L, r.y[1], r.y[2], r.y[4], r.y[5], r.k1);
    r.h = 1.0;
    r.last_cross = -INFINITY;
    const OutPtrs none{};
    int32_t st = 0;
    while (st == 0) {
        const int next = r.attempts + 1;
        const bool fault = next >= first && next <= last;
        st = ray::attempt<M>(fault ? bad : good, none, 1, r);
    }
    out.push_back(st);
    out.push_back(r.attempts);
    out.push_back(r.ncross);
    out.push_back(r.y[1]);
}

}  // namespace

int main() {
    const size_t width = 17;
    std::vector<double> in;
    double v;
    while (std::fread(&v, sizeof v, 1, stdin) == 1) in.push_back(v);
    if (in.size() % width) return 3;
    std::vector<double> out;
    for (size_t i = 0; i < in.size(); i += width) {
        const double* a = &in[i];
        const int m = static_cast<int>(a[0]);
        if (m == KERR) ray_case<KERR>(a, out);
        else if (m == EINASTO) ray_case<EINASTO>(a, out);
        else ray_case<CNFW>(a, out);
    }
    std::fwrite(out.data(), sizeof(double), out.size(), stdout);
    return 0;
}
