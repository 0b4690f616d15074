// Host driver for tests/test_vjp_host.py: runs the ray tracer's per-ray
// reverse-mode pieces (paper_2605_05635_amd/csrc/rt_vjp.h, compiled for the
// host from the same source) on rows of doubles read from stdin and writes
// the results to stdout.
//
//   vjp_driver rhs   row = metric chi m0 m1 m2 E L R th pR pth g0 g1 g2 g3
//     out: 10 values of rhs_vjp (R th pR pth E L chi m0 m1 m2), the same 10
//          from the dual-number Jacobian of rhs, and the 4 rows d1 d2 d4 d5.
//   vjp_driver step  row = metric chi m0 m1 m2 r_in r_out sig_in sig_out p
//                          E L R th pR pth h Ib w0 w1 w2 w3
//     The functional Phi = w . x(after the step) + Ib I(crossing) of one
//     step attempt of size h from x = (R, th, pR, pth) (the kernels' attempt()).
//     out: Phi, accepted, crossed, then 11 values of reverse_step
//          (R th pR pth E L chi m0 m1 m2 r_in).
//   vjp_driver root  row = y0 r2 r3 r4 r5 up0
//     The crossing root of theta's continuous extension with those
//     coefficients (ray::crossing_root).  out: s.
#include <cstdio>
#include <cstring>
#include <vector>

#include "rt_vjp.h"

using namespace rt;

namespace {

ImageConst consts(const double* a) {
    ImageConst c;
    std::memset(&c, 0, sizeof c);
    c.metric = static_cast<int32_t>(a[0]);
    c.chi = a[1];
    c.chi2 = a[1] * a[1];
    if (c.metric == EINASTO) c.inv_lam = a[2];
    if (c.metric == CNFW) {
        c.lam_c = a[2];
        c.inv_lam_c = a[3];
        c.eta_lc = a[4];
    }
    c.max_attempts = 1 << 30;
    c.rtol = c.atol = 1e-2;   // any attempt of the sizes used is accepted
    c.r_stop = 0.0;
    c.r_esc = 1e300;
    c.h0 = 1.0;
    c.nx = c.ny = 1;
    c.n_pix = 1;
    c.emission = 1;
    return c;
}

template <int M>
void rhs_case(const double* a, std::vector<double>& out) {
    const ImageConst c = consts(a);
    const ray::Hot k = ray::hot_of(c);
    const double E = a[5], L = a[6];
    const double x[4] = {a[7], a[8], a[9], a[10]};
    const double g[4] = {a[11], a[12], a[13], a[14]};
    double xb[4] = {0, 0, 0, 0}, Eb = 0, Lb = 0, pb[4] = {0, 0, 0, 0};
    vjp::rhs_vjp<M>(k, E, L, x, g, xb, Eb, Lb, pb);
    for (double v : xb) out.push_back(v);
    out.push_back(Eb);
    out.push_back(Lb);
    for (double v : pb) out.push_back(v);

    using D = Dual<10>;
    rt::Coeffs<D> kd;
    kd.chi = D::var(c.chi, 6);
    kd.chi2 = kd.chi * kd.chi;
    kd.inv_lam = D::var(c.inv_lam, 7);
    kd.lam_c = D::var(c.lam_c, 7);
    kd.inv_lam_c = D::var(c.inv_lam_c, 8);
    kd.eta_lc = D::var(c.eta_lc, 9);
    D d[6];
    ray::rhs<M>(kd, D::var(E, 4), D::var(L, 5), D::var(x[0], 0), D::var(x[1], 1),
                D::var(x[2], 2), D::var(x[3], 3), d);
    const int rows[4] = {1, 2, 4, 5};
    for (int j = 0; j < 10; ++j) {
        double v = 0.0;
        for (int r = 0; r < 4; ++r) v += g[r] * d[rows[r]].d[j];
        out.push_back(v);
    }
    for (int r = 0; r < 4; ++r) out.push_back(d[rows[r]].v);
}

template <int M>
void step_case(const double* a, std::vector<double>& out) {
    ImageConst c = consts(a);
    c.r_in = a[5];
    c.r_out = a[6];
    c.sigma_in = a[7];
    c.sigma_out = a[8];
    c.taper = (c.sigma_in > 0.0 && c.sigma_out > 0.0) ? 1 : 0;
    c.emis_pow = a[9];
    const ray::Hot k = ray::hot_of(c);
    const double E = a[10], L = a[11];
    const double x[4] = {a[12], a[13], a[14], a[15]};
    const double h = a[16], Ib = a[17];
    const double w[4] = {a[18], a[19], a[20], a[21]};

    ray::Ray r;
    std::memset(&r, 0, sizeof r);
    ray::set_constants(k.chi, E, L, r);
    r.y[1] = x[0];
    r.y[2] = x[1];
    r.y[4] = x[2];
    r.y[5] = x[3];
    ray::rhs<M>(k, E, L, r.y[1], r.y[2], r.y[4], r.y[5], r.k1);
    r.h = h;
    r.last_cross = -1e300;
    const OutPtrs none{};
    double rec[vjp::kRecDoubles] = {};
    ray::attempt<M>(k, none, 1, r, vjp::TapeStages{rec});
    const bool accepted = r.after_reject == 0;
    const bool crossed = r.ncross == 1;
    double phi = w[0] * r.y[1] + w[1] * r.y[2] + w[2] * r.y[4] + w[3] * r.y[5];
    if (crossed) {
        const double R = r.rc[0];
        const double g = ray::redshift<M>(k, R, E, L);
        phi += Ib * ray::disc_window(c, R, c.r_in) * g * g * g * std::pow(R, -c.emis_pow);
    }
    out.push_back(phi);
    out.push_back(accepted ? 1.0 : 0.0);
    out.push_back(crossed ? 1.0 : 0.0);
    double xb[4] = {w[0], w[1], w[2], w[3]};
    double Eb = 0, Lb = 0, pb[4] = {0, 0, 0, 0}, rinb = 0;
    vjp::reverse_step<M>(c, k, E, L, x, h, crossed ? 0 : -1, rec + vjp::kRecStages, Ib, xb, Eb,
                         Lb, pb, rinb);
    for (double v : xb) out.push_back(v);
    out.push_back(Eb);
    out.push_back(Lb);
    for (double v : pb) out.push_back(v);
    out.push_back(rinb);
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    const bool rhs_mode = !std::strcmp(argv[1], "rhs");
    const bool step_mode = !std::strcmp(argv[1], "step");
    const bool root_mode = !std::strcmp(argv[1], "root");
    if (!rhs_mode && !step_mode && !root_mode) return 2;
    const size_t width = rhs_mode ? 15 : step_mode ? 22 : 6;
    std::vector<double> in;
    double v;
    while (std::fread(&v, sizeof v, 1, stdin) == 1) in.push_back(v);
    if (in.size() % width) return 3;
    std::vector<double> out;
    for (size_t i = 0; i < in.size(); i += width) {
        const double* a = &in[i];
        const int m = static_cast<int>(a[0]);
        if (root_mode) {
            ray::DenseComp d;
            d.y0 = a[0];
            d.r2 = a[1];
            d.r3 = a[2];
            d.r4 = a[3];
            d.r5 = a[4];
            out.push_back(ray::crossing_root(d, a[5] != 0.0, ray::kHalfPi));
        } else if (rhs_mode) {
            if (m == KERR) rhs_case<KERR>(a, out);
            else if (m == EINASTO) rhs_case<EINASTO>(a, out);
            else rhs_case<CNFW>(a, out);
        } else {
            if (m == KERR) step_case<KERR>(a, out);
            else if (m == EINASTO) step_case<EINASTO>(a, out);
            else step_case<CNFW>(a, out);
        }
    }
    std::fwrite(out.data(), sizeof(double), out.size(), stdout);
    return 0;
}
