// rt_ray32.h -- the binary32 bulk of the mixed-precision trace.
//
// A ray starts in binary32: the right-hand side, the Dormand-Prince stages and
// the step controller run in single precision (at the image's tolerances, no
// tighter than the binary32 floor), while the state itself is carried as an
// unevaluated sum hi + lo of two floats updated by error-free addition, so the
// position accumulated over hundreds of steps keeps nearly binary64 accuracy.
// Crossings are located in binary64 on the step's continuous extension built
// from the compensated end points.  The ray leaves binary32
//   * at the first step that would end within r_zone (1.5 R_+) of the
//     horizon: that step and the rest of the ray run in binary64 (hand-off);
//   * when it has two trusted crossings (a lensed, near-critical ray) or more
//     than kMaxAccepted32 accepted steps: it is traced again entirely in
//     binary64 (rerun).
// Both are finished by the binary64 code of rt_ray.h in a second pass, so the
// binary32 pass stays free of binary64 steps (no divergence between the two
// arithmetics inside a wavefront, and its own register budget).
#pragma once

#include "rt_ray.h"

namespace rt {
namespace ray32 {

using namespace ray;

constexpr int32_t kHandOff = -1;       // continue in binary64 from the current state
constexpr int32_t kRerun = -2;         // trace again in binary64 from the screen
constexpr int32_t kRerunCrossings = 2;
constexpr int32_t kMaxAccepted32 = 1024;

struct Hot32 {
    float chi, chi2, inv_lam, lam_c, inv_lam_c, eta_lc;
    float rtol, atol;
    double r_stop, r_esc, r_zone;
    int32_t max_attempts;
};

__device__ __forceinline__ Hot32 hot32_of(const ImageConst& c) {
    Hot32 k;
    k.chi = static_cast<float>(c.chi);
    k.chi2 = static_cast<float>(c.chi2);
    k.inv_lam = static_cast<float>(c.inv_lam);
    k.lam_c = static_cast<float>(c.lam_c);
    k.inv_lam_c = static_cast<float>(c.inv_lam_c);
    k.eta_lc = static_cast<float>(c.eta_lc);
    k.rtol = static_cast<float>(c.rtol32);
    k.atol = static_cast<float>(c.atol32);
    k.r_stop = c.r_stop;
    k.r_esc = c.r_esc;
    k.r_zone = c.r_zone;
    k.max_attempts = c.max_attempts;
    return k;
}

struct Ray32 {
    float hi[6], lo[6];   // state T, R, theta, phi, p_R, p_theta as hi + lo
    float k1[6];
    float E, L;
    float h;
    int32_t attempts, accepted, ncross, after_reject;
    double lam, last_cross;
    double rc[3];
    int64_t pix;
};

// Error-free sum of a state component and an increment: (hi, lo) + d with the
// rounding error of hi + d (Knuth's two-sum) folded into lo, then renormalised
// so that |lo| stays below half an ulp of hi.
__device__ __forceinline__ void compensated_add(float hi, float lo, float d, float& nhi,
                                                float& nlo) {
    const float s = hi + d;
    const float bp = s - hi;
    const float err = (hi - (s - bp)) + (d - bp);
    const float l = lo + err;
    nhi = s + l;
    nlo = l - (nhi - s);
}

__device__ __forceinline__ double wide(float hi, float lo) {
    return static_cast<double>(hi) + static_cast<double>(lo);
}

template <int METRIC>
__device__ __forceinline__ void start_ray32(const ImageConst& c, const Hot32& k, int64_t pix,
                                            Ray32& r) {
    const ScreenDir n = screen_dir(c, pix);
    const double E = c.obs_N - c.obs_gTph_over_sq_gphph * n.nph;
    const double L = c.obs_sq_gphph * n.nph;
    const double y[6] = {0.0, c.r_obs, c.incl, 0.0, c.obs_sq_gRR * n.nR, c.obs_sq_gthth * n.nth};
    for (int i = 0; i < 6; ++i) {
        r.hi[i] = static_cast<float>(y[i]);
        r.lo[i] = static_cast<float>(y[i] - static_cast<double>(r.hi[i]));
    }
    r.E = static_cast<float>(E);
    r.L = static_cast<float>(L);
    rhs<METRIC>(k, r.E, r.L, r.hi[1], r.hi[2], r.hi[4], r.hi[5], r.k1);
    r.h = static_cast<float>(c.h0);
    r.lam = 0.0;
    r.last_cross = -INFINITY;
    r.rc[0] = r.rc[1] = r.rc[2] = 0.0;
    r.attempts = r.accepted = r.ncross = r.after_reject = 0;
    r.pix = pix;
}

// One binary32 step attempt.  Returns 0 while the ray runs, a final status,
// kHandOff (the state is left as before the attempt) or kRerun.
template <int METRIC>
__device__ __forceinline__ int32_t attempt32(const Hot32& k, const OutPtrs& o, int64_t n_pix,
                                             Ray32& r) {
    if (r.attempts >= k.max_attempts) return RAY_STEP_LIMIT;
    ++r.attempts;
    const float h = r.h;
    float ab[6], ae[6], ad[6];
    float k2[6], k3[6], k4[6], k5[6], kk[6], t[6];
    constexpr float f_a21 = a21, f_a31 = a31, f_a32 = a32, f_a41 = a41, f_a42 = a42,
                    f_a43 = a43, f_a51 = a51, f_a52 = a52, f_a53 = a53, f_a54 = a54,
                    f_a61 = a61, f_a62 = a62, f_a63 = a63, f_a64 = a64, f_a65 = a65;
    constexpr float f_b1 = b1, f_b3 = b3, f_b4 = b4, f_b5 = b5, f_b6 = b6;
    constexpr float f_e1 = e1, f_e3 = e3, f_e4 = e4, f_e5 = e5, f_e6 = e6, f_e7 = e7;
    constexpr float f_d1 = d1, f_d3 = d3, f_d4 = d4, f_d5 = d5, f_d6 = d6, f_d7 = d7;
    for (int i = 0; i < 6; ++i) {
        ab[i] = f_b1 * r.k1[i];
        ae[i] = f_e1 * r.k1[i];
        ad[i] = f_d1 * r.k1[i];
    }
#define RT_STAGE32(expr, out)                                                    \
    for (int i = 0; i < 6; ++i) t[i] = r.hi[i] + h * (expr);                      \
    rhs<METRIC>(k, r.E, r.L, t[1], t[2], t[4], t[5], out);
#define RT_ACC32(bb, ee, dd, kv)                                                 \
    for (int i = 0; i < 6; ++i) {                                                \
        ab[i] += bb * kv[i];                                                     \
        ae[i] += ee * kv[i];                                                     \
        ad[i] += dd * kv[i];                                                     \
    }
    RT_STAGE32(f_a21 * r.k1[i], k2)
    RT_STAGE32(f_a31 * r.k1[i] + f_a32 * k2[i], k3)
    RT_ACC32(f_b3, f_e3, f_d3, k3)
    RT_STAGE32(f_a41 * r.k1[i] + f_a42 * k2[i] + f_a43 * k3[i], k4)
    RT_ACC32(f_b4, f_e4, f_d4, k4)
    RT_STAGE32(f_a51 * r.k1[i] + f_a52 * k2[i] + f_a53 * k3[i] + f_a54 * k4[i], k5)
    RT_ACC32(f_b5, f_e5, f_d5, k5)
    RT_STAGE32(f_a61 * r.k1[i] + f_a62 * k2[i] + f_a63 * k3[i] + f_a64 * k4[i] + f_a65 * k5[i], kk)
    RT_ACC32(f_b6, f_e6, f_d6, kk)
#undef RT_STAGE32
#undef RT_ACC32
    float nhi[6], nlo[6];
    for (int i = 0; i < 6; ++i) compensated_add(r.hi[i], r.lo[i], h * ab[i], nhi[i], nlo[i]);
    rhs<METRIC>(k, r.E, r.L, nhi[1], nhi[2], nhi[4], nhi[5], kk);   // k7
    float acc = 0.0f;
    for (int i = 0; i < 6; ++i) {
        ae[i] += f_e7 * kk[i];
        ad[i] += f_d7 * kk[i];
        const float sc = k.atol + k.rtol * fmaxf(fabsf(r.hi[i]), fabsf(nhi[i]));
        const float q = h * ae[i] * dm::recip(sc);
        acc += q * q;
    }
    const float err2 = acc * (1.0f / 6.0f);
    const float grow = 0.9f * dm::rpow_tenth(fminf(fmaxf(err2, 1e-12f), 1e12f));
    if (!(err2 < 1.0f)) {
        const bool finite = __builtin_isfinite(err2);
        r.h = h * (finite ? fmaxf(0.2f, grow) : 0.2f);
        // as in binary64; a ray that stays non-finite in binary32 is traced
        // again in binary64, which decides its fate
        r.after_reject = finite ? 1 : (r.after_reject | 1) + 2;
        return r.after_reject >= 2 * kNonfiniteRun + 1 ? kRerun : 0;
    }
    // A step into the horizon zone goes to binary64, with the rest of the ray.
    if (wide(nhi[1], nlo[1]) < k.r_zone) return kHandOff;
    float factor = err2 == 0.0f ? 10.0f : fminf(10.0f, grow);
    if (r.after_reject) factor = fminf(1.0f, factor);
    r.after_reject = 0;

    // Equatorial crossing, located in binary64 on the continuous extension
    // through the compensated end points.
    const double th0 = wide(r.hi[2], r.lo[2]), th1 = wide(nhi[2], nlo[2]);
    const double band0 = equator_band(th0);
    const double band1 = equator_band(th1);
    if (band0 != band1) {
        const Passage ps = passage_of(band0, band1);
        const double hd = static_cast<double>(h);
        auto dense = [&](int i) {
            DenseComp d;
            d.y0 = wide(r.hi[i], r.lo[i]);
            d.r2 = wide(nhi[i], nlo[i]) - d.y0;
            d.r3 = hd * static_cast<double>(r.k1[i]) - d.r2;
            d.r4 = d.r2 - hd * static_cast<double>(kk[i]) - d.r3;
            d.r5 = hd * static_cast<double>(ad[i]);
            return d;
        };
        const double s = crossing_root(dense(2), ps.up0, ps.th_eq);
        const double Rc = dense(1).at(s);
        const double pthc = dense(5).at(s);
        const double lc = r.lam + s * hd;
        if (fabs(pthc) >= 1e-12 * Rc * Rc && (lc - r.last_cross) >= 1e-10) {
            const int n = r.ncross;
            if (n < 3) {
                const int64_t off = static_cast<int64_t>(n) * n_pix + r.pix;
                r.rc[0] = n == 0 ? Rc : r.rc[0];
                r.rc[1] = n == 1 ? Rc : r.rc[1];
                r.rc[2] = n == 2 ? Rc : r.rc[2];
                if (o.r_em) o.r_em[off] = Rc;
                if (o.phi_em) o.phi_em[off] = dense(3).at(s) + ps.phi_shift;
                if (o.t_em) o.t_em[off] = dense(0).at(s);
            }
            if (r.ncross < 255) ++r.ncross;
            r.last_cross = lc;
        }
    }
    for (int i = 0; i < 6; ++i) {
        r.hi[i] = nhi[i];
        r.lo[i] = nlo[i];
        r.k1[i] = kk[i];
    }
    r.lam += static_cast<double>(h);
    r.h = h * factor;
    ++r.accepted;
    if (r.ncross >= kRerunCrossings || r.accepted > kMaxAccepted32) return kRerun;
    const double R = static_cast<double>(r.hi[1]);
    if (R <= k.r_stop) return RAY_CAPTURED;
    if (R >= k.r_esc) return RAY_ESCAPED;
    return 0;
}

// The binary64 ray at a binary32 ray's current state (all but k1).
__device__ __forceinline__ void widen(const ImageConst& c, const Ray32& r, Ray& w) {
    const ScreenDir n = screen_dir(c, r.pix);
    ray::set_constants(c.chi, c.obs_N - c.obs_gTph_over_sq_gphph * n.nph, c.obs_sq_gphph * n.nph, w);
    for (int i = 0; i < 6; ++i) w.y[i] = wide(r.hi[i], r.lo[i]);
    w.h = static_cast<double>(r.h);
    w.lam = r.lam;
    w.last_cross = r.last_cross;
    w.rc[0] = r.rc[0];
    w.rc[1] = r.rc[1];
    w.rc[2] = r.rc[2];
    w.attempts = r.attempts;
    w.ncross = r.ncross;
    w.after_reject = r.after_reject;
    w.pix = r.pix;
}

// Hand-off record of a ray in binary64 (kRecord doubles): state, step size,
// affine parameter, last crossing, the three crossing radii, E, l, attempt
// and crossing counts, the reject flag, the pixel, and whether the ray is to
// be traced again from the screen (1) or continued (0).
constexpr int kRecord = 20;

__device__ __forceinline__ void store_record(double* rec, const Ray& w) {
    for (int i = 0; i < 6; ++i) rec[i] = w.y[i];
    rec[6] = w.h;
    rec[7] = w.lam;
    rec[8] = w.last_cross;
    rec[9] = w.rc[0];
    rec[10] = w.rc[1];
    rec[11] = w.rc[2];
    rec[12] = w.E;
    rec[13] = w.L;
    rec[14] = static_cast<double>(w.attempts);
    rec[15] = static_cast<double>(w.ncross);
    rec[16] = static_cast<double>(w.after_reject);
    rec[17] = static_cast<double>(w.pix);
    rec[18] = 0.0;
    rec[19] = 0.0;
}

__device__ __forceinline__ void store_rerun(double* rec, int64_t pix) {
    for (int i = 0; i < kRecord; ++i) rec[i] = 0.0;
    rec[17] = static_cast<double>(pix);
    rec[18] = 1.0;
}

template <int METRIC>
__device__ __forceinline__ void load_record(const ImageConst& c, const Hot& k64, const double* rec,
                                            Ray& w) {
    const int64_t pix = static_cast<int64_t>(rec[17]);
    if (rec[18] != 0.0) {
        start_ray<METRIC>(c, k64, pix, w);
        return;
    }
    for (int i = 0; i < 6; ++i) w.y[i] = rec[i];
    w.h = rec[6];
    w.lam = rec[7];
    w.last_cross = rec[8];
    w.rc[0] = rec[9];
    w.rc[1] = rec[10];
    w.rc[2] = rec[11];
    ray::set_constants(k64.chi, rec[12], rec[13], w);
    w.attempts = static_cast<int32_t>(rec[14]);
    w.ncross = static_cast<int32_t>(rec[15]);
    w.after_reject = static_cast<int32_t>(rec[16]);
    w.pix = pix;
    rhs<METRIC>(k64, w.E, w.L, w.y[1], w.y[2], w.y[4], w.y[5], w.k1);
}

}  // namespace ray32
}  // namespace rt
