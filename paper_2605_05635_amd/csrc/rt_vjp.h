// rt_vjp.h -- reverse mode of one ray's computed discrete map: the adjoint of
// the right-hand side, of one accepted Dormand-Prince step (with the
// equatorial-crossing root located on its continuous extension), and of the
// emission of a crossing.  Host and device.
//
// The map differentiated is the one the trace computes, with its discrete
// decisions held fixed: the sizes of the accepted steps, which attempts were
// accepted, the step in which each crossing was found, the termination step,
// and the indicator parts of the disc window and of the emitter's existence.
// Only the T and phi components of the state never feed back into anything
// the intensity depends on, so the adjoint state is (R, theta, p_R, p_theta)
// together with the ray's constants E and l.
#pragma once

#include "rt_ray.h"

namespace rt {
namespace vjp {

using namespace ray;

// Per-ray parameter adjoints, in this order: spin chi, the three mass-function
// constants (Einasto: 1/lambda_E; cored NFW: lambda_c, 1/lambda_c,
// eta lambda_c), the disc window's inner edge, the five observer-frame
// constants of the screen map (N_o, g_Tphi/sqrt(g_phiphi), sqrt(g_phiphi),
// sqrt(g_RR), sqrt(g_thth) at the observer) and the inclination.
enum Prim {
    P_CHI = 0,
    P_M0,
    P_M1,
    P_M2,
    P_RIN,
    P_OBS_N,
    P_OBS_TPH,
    P_OBS_PH,
    P_OBS_R,
    P_OBS_TH,
    P_INCL,
    kPrims
};

// One accepted step on the tape: the state (R, theta, p_R, p_theta) at its
// start, its size, the index (0, 1, 2) of the crossing it recorded or -1, and
// its six stage derivatives' (R, theta, p_R, p_theta) rows (record[6 + 4j + i]
// for k_{j+1}), so that the reverse pass need not recompute them.
constexpr int kRecDoubles = 30;
constexpr int kRecStages = 6;   // offset of the stage derivatives

// Attempt sink that writes the stage derivatives into the tape record `rec`
// (always a writable record: a branch here would keep registers live across
// every stage).
struct TapeStages {
    double* rec;
    __host__ __device__ __forceinline__ void operator()(int j, const double* kj) const {
        double2* q = reinterpret_cast<double2*>(rec + kRecStages + 4 * j);
        q[0] = double2{kj[1], kj[2]};
        q[1] = double2{kj[4], kj[5]};
    }
};

// A checkpoint of a ray between two accepted steps: everything `attempt`
// reads besides the image constants, the photon's E and l (recomputed from
// the pixel) and k1 (the right-hand side at y, recomputed bit for bit):
// y[6], h, lam, last_cross, rc[3], and as exact doubles attempts, the
// accepted-step index, after_reject and ncross: 16 doubles.
constexpr int kCkptDoubles = 16;

__host__ __device__ __forceinline__ void store_checkpoint(double* slot, const Ray& r, int32_t acc) {
    double2* q = reinterpret_cast<double2*>(slot);
    q[0] = double2{r.y[0], r.y[1]};
    q[1] = double2{r.y[2], r.y[3]};
    q[2] = double2{r.y[4], r.y[5]};
    q[3] = double2{r.h, r.lam};
    q[4] = double2{r.last_cross, r.rc[0]};
    q[5] = double2{r.rc[1], r.rc[2]};
    q[6] = double2{static_cast<double>(r.attempts), static_cast<double>(acc)};
    q[7] = double2{static_cast<double>(r.after_reject), static_cast<double>(r.ncross)};
}

// Restores the checkpoint `slot` into r (pixel pix, constants E, l) for the
// metric's right-hand side; returns its accepted-step index.
template <int METRIC>
__host__ __device__ __forceinline__ int32_t load_checkpoint(const double* slot, const Hot& k,
                                                            double E, double L, int64_t pix,
                                                            Ray& r) {
    const double2* q = reinterpret_cast<const double2*>(slot);
    const double2 a = q[0], b = q[1], c = q[2], d = q[3], e = q[4], f = q[5], g = q[6],
                  h = q[7];
    r.y[0] = a.x;
    r.y[1] = a.y;
    r.y[2] = b.x;
    r.y[3] = b.y;
    r.y[4] = c.x;
    r.y[5] = c.y;
    r.h = d.x;
    r.lam = d.y;
    r.last_cross = e.x;
    r.rc[0] = e.y;
    r.rc[1] = f.x;
    r.rc[2] = f.y;
    r.attempts = static_cast<int32_t>(g.x);
    r.after_reject = static_cast<int32_t>(h.x);
    r.ncross = static_cast<int32_t>(h.y);
    set_constants(k.chi, E, L, r);
    r.pix = pix;
    rhs<METRIC>(k, E, L, r.y[1], r.y[2], r.y[4], r.y[5], r.k1);
    return static_cast<int32_t>(g.y);
}

// F(R), dF/dR (mass_function) and the reverse mode of both: mass_eval gives
// the values and keeps what the reverse pass needs; mass_vjp adds the
// cotangents (Fb, dFb) times the derivatives along R to Rb and along the
// metric's mass constants to mb[0..2] (Einasto: 1/lambda_E; cored NFW:
// lambda_c, 1/lambda_c, eta lambda_c).  Written out line by line against the
// forward formulas of mass_function.
template <int METRIC>
struct MassTape {
    double F, dF;
    double a[8];   // forward intermediates (metric-specific)
};

template <int METRIC>
__host__ __device__ __forceinline__ void mass_eval(const Hot& k, double R, MassTape<METRIC>& t) {
    if constexpr (METRIC == KERR) {
        t.F = 2.0 * R;
        t.dF = 2.0;
    } else if constexpr (METRIC == EINASTO) {
        const double x = R * k.inv_lam;
        const double e = dm::exp(-x);
        const double mu = 1.0 - e * (1.0 + x * (1.0 + 0.5 * x));
        const double dmu = 0.5 * e * x * x * k.inv_lam;
        t.F = 2.0 * R * mu;
        t.dF = 2.0 * (mu + R * dmu);
        t.a[0] = x;
        t.a[1] = e;
        t.a[2] = mu;
        t.a[3] = dmu;
    } else {
        const double Rl = R + k.lam_c;
        const double inv = dm::recip1(R * Rl);
        const double iR = Rl * inv;
        const double iRl = R * inv;
        const double u = R * k.inv_lam_c;
        const double lg = dm::log1p_fast(u);
        const double P = iRl - 2.0 * iR * lg;
        const double Q = 2.0 * iR * (iR * lg - iRl) - iRl * iRl;
        const double ex = k.eta_lc * P;
        const double dex = k.eta_lc * Q;
        const double em1 = dm::expm1(ex, METRIC == CNFW_NEAR);
        t.F = R * (2.0 - R * em1);
        t.dF = 2.0 - R * (2.0 * em1 + R * (em1 + 1.0) * dex);
        t.a[0] = iR;
        t.a[1] = iRl;
        t.a[2] = u;
        t.a[3] = lg;
        t.a[4] = P;
        t.a[5] = Q;
        t.a[6] = em1;
        t.a[7] = dex;
    }
}

template <int METRIC>
__host__ __device__ __forceinline__ void mass_vjp(const Hot& k, double R,
                                                  const MassTape<METRIC>& t, double Fb,
                                                  double dFb, double& Rb, double mb[3]) {
    if constexpr (METRIC == KERR) {
        Rb += 2.0 * Fb;
    } else if constexpr (METRIC == EINASTO) {
        const double x = t.a[0], e = t.a[1], mu = t.a[2], dmu = t.a[3];
        // F = 2 R mu, dF = 2 (mu + R dmu)
        const double b_mu = 2.0 * R * Fb + 2.0 * dFb;
        const double b_dmu = 2.0 * R * dFb;
        Rb += 2.0 * mu * Fb + 2.0 * dmu * dFb;
        // dmu = e x^2 inv_lam / 2
        double b_e = 0.5 * b_dmu * x * x * k.inv_lam;
        double b_x = b_dmu * e * x * k.inv_lam;
        double b_inv = 0.5 * b_dmu * e * x * x;
        // mu = 1 - e (1 + x + x^2/2)
        b_e -= b_mu * (1.0 + x * (1.0 + 0.5 * x));
        b_x -= b_mu * e * (1.0 + x);
        // e = exp(-x), x = R inv_lam
        b_x -= b_e * e;
        Rb += b_x * k.inv_lam;
        b_inv += b_x * R;
        mb[0] += b_inv;
    } else {
        const double iR = t.a[0], iRl = t.a[1], u = t.a[2], lg = t.a[3], P = t.a[4],
                     Q = t.a[5], em1 = t.a[6], dex = t.a[7];
        // F = 2R - R^2 em1;  dF = 2 - 2R em1 - R^2 (em1 + 1) dex
        Rb += Fb * (2.0 - 2.0 * R * em1) + dFb * (-2.0 * em1 - 2.0 * R * (em1 + 1.0) * dex);
        const double b_em1 = -Fb * R * R + dFb * (-2.0 * R - R * R * dex);
        const double b_dex = -dFb * R * R * (em1 + 1.0);
        // em1 = expm1(ex)
        const double b_ex = b_em1 * (em1 + 1.0);
        // dex = eta_lc Q, ex = eta_lc P
        double b_eta = b_dex * Q + b_ex * P;
        const double b_Q = b_dex * k.eta_lc;
        const double b_P = b_ex * k.eta_lc;
        // Q = 2 iR^2 lg - 2 iR iRl - iRl^2;  P = iRl - 2 iR lg
        const double b_iR = b_Q * (4.0 * iR * lg - 2.0 * iRl) - 2.0 * b_P * lg;
        const double b_lg = b_Q * 2.0 * iR * iR - 2.0 * b_P * iR;
        const double b_iRl = b_Q * (-2.0 * iR - 2.0 * iRl) + b_P;
        // lg = log1p(u), u = R inv_lam_c
        const double b_u = b_lg * dm::recip1(1.0 + u);
        Rb += b_u * k.inv_lam_c;
        const double b_ilc = b_u * R;
        // iR = 1/R, iRl = 1/(R + lam_c)
        Rb += -b_iR * iR * iR;
        const double b_Rl = -b_iRl * iRl * iRl;
        Rb += b_Rl;
        mb[0] += b_Rl;     // lambda_c
        mb[1] += b_ilc;    // 1/lambda_c
        mb[2] += b_eta;    // eta lambda_c
    }
}

// Reverse mode of the R, theta, p_R, p_theta rows of rhs (d[1], d[2], d[4],
// d[5]) at x = (R, theta, p_R, p_theta): for the cotangent g of those rows,
// adds g^T (d rows / d x) to xb, the derivatives along E and l to Eb and Lb,
// and those along chi and the mass constants to pb[0..3].  The forward
// quantities are those of rhs; each adjoint line below undoes one of them.
template <int METRIC>
__host__ __device__ __forceinline__ void rhs_vjp(const Hot& k, double E, double L,
                                                 const double x[4], const double g[4],
                                                 double xb[4], double& Eb, double& Lb,
                                                 double pb[4]) {
    const double R = x[0], th = x[1], pR = x[2], pth = x[3];
    double s, co;
    dm::sincos(th, &s, &co);
    MassTape<METRIC> mt;
    mass_eval<METRIC>(k, R, mt);
    const double F = mt.F, dF = mt.dF;
    const double R2 = R * R;
    const double R2c = R2 + k.chi2;
    const double cc = co * co;
    const double Sig = R2 + k.chi2 * cc;
    const double Del = R2c - F;
    const double dDel = 2.0 * R - dF;
    const double iS = rcp(Sig);
    const double iD = rcp(Del);
    const double is = rcp(s);
    const double P = R2c * E - k.chi * L;
    const double PiD = P * iD;
    const double Lis = L * is;
    const double Lis2 = Lis * is;
    const double chiE = k.chi * E;
    const double W = Lis - chiE * s;
    const double pR2 = pR * pR;
    const double N = Del * pR2 + pth * pth - P * PiD + W * W;
    const double dN = dDel * (pR2 + PiD * PiD) - 4.0 * R * E * PiD;
    const double A5 = Lis2 + chiE;
    const double Q5 = W * A5 - k.chi2 * s * N * iS;
    const double Q4 = N * R * iS - 0.5 * dN;
    const double gR = g[0], gth = g[1], gpR = g[2], gpth = g[3];

    // d5 = co iS Q5
    const double bQ5 = gpth * co * iS;
    double b_co = gpth * iS * Q5;
    double b_iS = gpth * co * Q5;
    double b_W = bQ5 * A5;
    double b_Lis2 = bQ5 * W;
    double b_chiE = bQ5 * W;
    double b_chi2 = -bQ5 * s * N * iS;
    double b_s = -bQ5 * k.chi2 * N * iS;
    double b_N = -bQ5 * k.chi2 * s * iS;
    b_iS -= bQ5 * k.chi2 * s * N;
    // d4 = Q4 iS
    const double bQ4 = gpR * iS;
    b_iS += gpR * Q4 + bQ4 * N * R;
    b_N += bQ4 * R * iS;
    double b_R = bQ4 * N * iS;
    const double b_dN = -0.5 * bQ4;
    // d2 = pth iS
    double b_pth = gth * iS;
    b_iS += gth * pth;
    // d1 = Del pR iS
    double b_Del = gR * pR * iS;
    double b_pR = gR * Del * iS;
    b_iS += gR * Del * pR;
    // dN = dDel (pR^2 + PiD^2) - 4 R E PiD
    double b_dDel = b_dN * (pR2 + PiD * PiD);
    double b_pR2 = b_dN * dDel;
    double b_PiD = b_dN * (2.0 * dDel * PiD - 4.0 * R * E);
    b_R -= 4.0 * b_dN * E * PiD;
    double b_E = -4.0 * b_dN * R * PiD;
    // N = Del pR^2 + pth^2 - P PiD + W^2
    b_Del += b_N * pR2;
    b_pR2 += b_N * Del;
    b_pth += 2.0 * b_N * pth;
    double b_P = -b_N * PiD;
    b_PiD -= b_N * P;
    b_W += 2.0 * b_N * W;
    b_pR += 2.0 * pR * b_pR2;
    // W = Lis - chiE s
    double b_Lis = b_W;
    b_chiE -= b_W * s;
    b_s -= b_W * chiE;
    // chiE = chi E
    double b_chi = b_chiE * E;
    b_E += b_chiE * k.chi;
    // Lis2 = Lis is, Lis = L is
    b_Lis += b_Lis2 * is;
    double b_is = b_Lis2 * Lis;
    double b_L = b_Lis * is;
    b_is += b_Lis * L;
    // PiD = P iD
    b_P += b_PiD * iD;
    const double b_iD = b_PiD * P;
    // P = R2c E - chi L
    double b_R2c = b_P * E;
    b_E += b_P * R2c;
    b_chi -= b_P * L;
    b_L -= b_P * k.chi;
    // reciprocals
    b_s -= b_is * is * is;
    b_Del -= b_iD * iD * iD;
    const double b_Sig = -b_iS * iS * iS;
    // dDel = 2R - dF, Del = R2c - F
    b_R += 2.0 * b_dDel;
    const double b_dF = -b_dDel;
    b_R2c += b_Del;
    const double b_F = -b_Del;
    // Sig = R2 + chi2 cc, R2c = R2 + chi2, R2 = R R, cc = co co
    double b_R2 = b_Sig + b_R2c;
    b_chi2 += b_Sig * cc + b_R2c;
    b_co += 2.0 * co * b_Sig * k.chi2;
    b_R += 2.0 * R * b_R2;
    // (s, co) = (sin th, cos th)
    const double b_th = b_s * co - b_co * s;
    // mass function
    mass_vjp<METRIC>(k, R, mt, b_F, b_dF, b_R, pb + 1);
    // chi2 = chi^2
    b_chi += 2.0 * k.chi * b_chi2;

    xb[0] += b_R;
    xb[1] += b_th;
    xb[2] += b_pR;
    xb[3] += b_pth;
    Eb += b_E;
    Lb += b_L;
    pb[0] += b_chi;
}

// Intensity of one crossing, I_n = w(R) g^3 R^(-p) (eqs. (89)-(91) and the
// window of eq. (77) or eqs. (85)-(86)), and its derivatives: with the
// cotangent Ib of I_n, sets Rb and adds to Eb, Lb, pb[0..3] (chi and the mass
// constants) and rinb (the window's inner edge).  Dual numbers along
// (R, E, l, chi, mass constants, r_in).
template <int METRIC>
__host__ __device__ __forceinline__ double emission_vjp(const ImageConst& c, double R, double E,
                                                        double L, double Ib, double& Rb,
                                                        double& Eb, double& Lb, double pb[4],
                                                        double& rinb) {
    using D = Dual<8>;
    Coeffs<D> kd;
    kd.chi = D::var(c.chi, 3);
    kd.chi2 = kd.chi * kd.chi;
    if constexpr (METRIC == EINASTO) {
        kd.inv_lam = D::var(c.inv_lam, 4);
    } else if constexpr (is_cnfw(METRIC)) {
        kd.lam_c = D::var(c.lam_c, 4);
        kd.inv_lam_c = D::var(c.inv_lam_c, 5);
        kd.eta_lc = D::var(c.eta_lc, 6);
    }
    const D Rd = D::var(R, 0);
    const D g = redshift<METRIC>(kd, Rd, D::var(E, 1), D::var(L, 2));
    const D I = disc_window(c, Rd, D::var(c.r_in, 7)) * g * g * g * pow(Rd, -c.emis_pow);
    Rb = Ib * I.d[0];
    Eb += Ib * I.d[1];
    Lb += Ib * I.d[2];
    for (int j = 0; j < 4; ++j) pb[j] += Ib * I.d[3 + j];
    rinb += Ib * I.d[7];
    return I.v;
}

// Whether crossing radius R contributes a non-zero intensity (hence a
// non-zero derivative): inside the window and with a timelike emitter.
template <int METRIC>
__host__ __device__ __forceinline__ bool emits(const ImageConst& c, const Hot& k, double R,
                                               double E, double L) {
    return disc_window(c, R, c.r_in) != 0.0 && redshift<METRIC>(k, R, E, L) != 0.0;
}

// Reverse of one accepted step of size h from x0 = (R, theta, p_R, p_theta).
// On entry xb is the adjoint of the state after the step, on return the
// adjoint of x0.  If the step recorded a crossing (cross >= 0), its
// intensity's cotangent Ib enters through the crossing radius, located on the
// continuous extension at the root s* of theta(s) = theta_eq (pi/2, or the
// equator's value beyond a pole): with
//   y(s) = y0 + h sum_j beta_j(s) k_j,
//   beta_j = (3s^2 - 2s^3) b_j + [j=1] s(1-s)^2 - [j=7] s^2(1-s) + s^2(1-s)^2 d_j,
// R_c = R(s*) moves by dR - (R'(s*)/theta'(s*)) dtheta (implicit function
// theorem), so the R and theta rows receive the cotangents Rb and
// -Rb R'/theta'.  The stage derivatives kin[4j + i] are the forward step's
// (its tape record); the stage inputs are formed from them exactly as the
// forward step forms them, then the stages are reversed from the last to the
// first.
template <int METRIC>
__host__ __device__ __forceinline__ void reverse_step(const ImageConst& c, const Hot& k, double E,
                                                      double L, const double x0[4], double h,
                                                      int cross, const double* kin, double Ib,
                                                      double xb[4], double& Eb, double& Lb,
                                                      double pb[4], double& rinb) {
    constexpr double A[6][5] = {{0.0, 0.0, 0.0, 0.0, 0.0},
                                {a21, 0.0, 0.0, 0.0, 0.0},
                                {a31, a32, 0.0, 0.0, 0.0},
                                {a41, a42, a43, 0.0, 0.0},
                                {a51, a52, a53, a54, 0.0},
                                {a61, a62, a63, a64, a65}};
    constexpr double B[7] = {b1, 0.0, b3, b4, b5, b6, 0.0};
    constexpr double Dc[7] = {d1, 0.0, d3, d4, d5, d6, d7};
    auto f = [&](const double* xin, double* out) {
        double d[6];
        rhs<METRIC>(k, E, L, xin[0], xin[1], xin[2], xin[3], d);
        out[0] = d[1];
        out[1] = d[2];
        out[2] = d[4];
        out[3] = d[5];
    };
    // The forward step's stage derivatives.
    double kv[6][4], ab[4];
    for (int j = 0; j < 6; ++j)
        for (int i = 0; i < 4; ++i) kv[j][i] = kin[4 * j + i];
    double yn[4];
    for (int i = 0; i < 4; ++i) {
        ab[i] = b1 * kv[0][i];
        ab[i] += b3 * kv[2][i];
        ab[i] += b4 * kv[3][i];
        ab[i] += b5 * kv[4][i];
        ab[i] += b6 * kv[5][i];
        yn[i] = x0[i] + h * ab[i];
    }

    double kb[6][4];
    for (int j = 0; j < 6; ++j)
        for (int i = 0; i < 4; ++i) kb[j][i] = 0.0;
    double cR = 0.0, cth = 0.0;
    if (cross >= 0) {
        double k7[4];
        f(yn, k7);
        DenseComp dc[2];   // R, theta
        for (int i = 0; i < 2; ++i) {
            double ad = d1 * kv[0][i];
            ad += d3 * kv[2][i];
            ad += d4 * kv[3][i];
            ad += d5 * kv[4][i];
            ad += d6 * kv[5][i];
            ad += d7 * k7[i];
            dc[i].y0 = x0[i];
            dc[i].r2 = yn[i] - x0[i];
            dc[i].r3 = h * kv[0][i] - dc[i].r2;
            dc[i].r4 = dc[i].r2 - h * k7[i] - dc[i].r3;
            dc[i].r5 = h * ad;
        }
        const Passage ps = passage_of(equator_band(x0[1]), equator_band(yn[1]));
        const double s = crossing_root(dc[1], ps.up0, ps.th_eq);
        const double Rc = dc[0].at(s);
        double Rb = 0.0;
        emission_vjp<METRIC>(c, Rc, E, L, Ib, Rb, Eb, Lb, pb, rinb);
        if (Rb != 0.0) {
            double slope[2];
            for (int i = 0; i < 2; ++i) {
                const double c1 = dc[i].r2 + dc[i].r3;
                const double c2 = dc[i].r4 + dc[i].r5 - dc[i].r3;
                const double c3 = -dc[i].r4 - 2.0 * dc[i].r5;
                const double c4 = dc[i].r5;
                slope[i] = c1 + s * (2.0 * c2 + s * (3.0 * c3 + s * 4.0 * c4));
            }
            cR = Rb;
            cth = -Rb * slope[0] / slope[1];
            const double s1 = 1.0 - s;
            const double B5 = s * s * (3.0 - 2.0 * s);
            const double S2 = s * s * s1 * s1;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                const double beta = B5 * B[j] + S2 * Dc[j] + (j == 0 ? s * s1 * s1 : 0.0);
                kb[j][0] = h * beta * cR;
                kb[j][1] = h * beta * cth;
            }
            const double beta7 = S2 * Dc[6] - s * s * s1;
            const double g7[4] = {h * beta7 * cR, h * beta7 * cth, 0.0, 0.0};
            rhs_vjp<METRIC>(k, E, L, yn, g7, xb, Eb, Lb, pb);
        }
    }
    // yn = x0 + h sum_j b_j k_j
    double x0b[4];
    for (int i = 0; i < 4; ++i) {
        x0b[i] = xb[i];
        for (int j = 0; j < 6; ++j) kb[j][i] += h * B[j] * xb[i];
    }
    x0b[0] += cR;
    x0b[1] += cth;
    // stages 6..2: Y_j = x0 + h sum_{l<j} a_jl k_l, k_j = f(Y_j)
#pragma unroll
    for (int j = 5; j >= 1; --j) {
        double Y[4], Yb[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < 4; ++i) {
            double acc = 0.0;
            for (int l = 0; l < j; ++l) acc += A[j][l] * kv[l][i];
            Y[i] = x0[i] + h * acc;
        }
        rhs_vjp<METRIC>(k, E, L, Y, kb[j], Yb, Eb, Lb, pb);
        for (int i = 0; i < 4; ++i) {
            x0b[i] += Yb[i];
            for (int l = 0; l < j; ++l) kb[l][i] += h * A[j][l] * Yb[i];
        }
    }
    rhs_vjp<METRIC>(k, E, L, x0, kb[0], x0b, Eb, Lb, pb);
    for (int i = 0; i < 4; ++i) xb[i] = x0b[i];
}

}  // namespace vjp
}  // namespace rt
