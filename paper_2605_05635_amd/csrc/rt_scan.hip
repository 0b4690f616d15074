// rt_scan.hip -- parameter scans of the spacetimes (Sec. 2): per point, the
// outer horizon (eq. (33)), the ergosurface radius at one polar angle, and the
// extremal spin with its radius.  One wavefront per point: the searches of
// rt_scan.h with their grids split into 64 contiguous runs, one per lane; the
// wavefront keeps the interval the serial search would have kept (the first
// from the top for a root, the first minimum of least value for the extremal
// spin) and refines it exactly as the serial search does, so the results are
// the same bits as rt_scan.h's.
#include "rt.h"
#include "rt_scan.h"

namespace rt {
namespace {

using scan::delta;

// The bracket the serial largest_root would bisect, found by 64 lanes; the
// refinement is largest_root's own.
__device__ bool largest_root_wave(const ImageConst& c, double a2, double* root) {
    const double top = 50.0, step = 1e-2;
    const int lane = __lane_id();
    double D_top, dD_top;
    delta(c, a2, top, &D_top, &dD_top);
    if (!(D_top > 0.0)) return false;
    int n = 0;   // intervals k = 1..n, as the serial loop's condition
    while (top - (n + 1) * step >= 0.05 - 1e-12) ++n;
    const int per = (n + 63) / 64;
    const int k0 = 1 + lane * per, k1 = k0 + per - 1 < n ? k0 + per - 1 : n;
    int found = 0;
    double fa = 0.0, fb = 0.0;
    if (k0 <= k1) {
        double D_hi, dD_hi;
        delta(c, a2, top - (k0 - 1) * step, &D_hi, &dD_hi);
        for (int k = k0; k <= k1 && !found; ++k) {
            const double hi = top - (k - 1) * step, lo = top - k * step;
            double D_lo, dD_lo;
            delta(c, a2, lo, &D_lo, &dD_lo);
            double a = lo;
            bool bracket = D_lo <= 0.0;
            if (!bracket && dD_lo < 0.0 && dD_hi > 0.0) {
                double u = lo, v = hi;
                for (int it = 0; it < 200; ++it) {
                    const double m = 0.5 * (u + v);
                    if (m <= u || m >= v) break;
                    double Dm, dDm;
                    delta(c, a2, m, &Dm, &dDm);
                    if (dDm < 0.0) u = m; else v = m;
                }
                double Dm, dDm;
                delta(c, a2, 0.5 * (u + v), &Dm, &dDm);
                if (Dm <= 0.0) {
                    a = 0.5 * (u + v);
                    bracket = true;
                }
            }
            if (bracket) {
                found = 1;
                fa = a;
                fb = hi;
            }
            D_hi = D_lo;
            dD_hi = dD_lo;
        }
    }
    const unsigned long long m = __ballot(found);
    if (m == 0ull) return false;
    const int src = __ffsll(static_cast<long long>(m)) - 1;   // the topmost run with a bracket
    double a = __shfl(fa, src), b = __shfl(fb, src);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (a + b);
        if (mid <= a || mid >= b) break;
        double Dm, dDm;
        delta(c, a2, mid, &Dm, &dDm);
        if (Dm > 0.0) b = mid; else a = mid;
    }
    *root = 0.5 * (a + b);
    return true;
}

// extremal_spin of rt_scan.h with its grid split over the lanes: each lane
// keeps its first minimum of least value, the wavefront the least over the
// lanes (the lowest lane among equals: the serial scan's first).
__device__ bool extremal_spin_wave(const ImageConst& c, double* chi_e, double* r_e) {
    const double step = 1e-3;
    const int lane = __lane_id();
    int n = 0;   // intervals k = 1..n: the serial loop runs while a < 50
    while (0.01 + static_cast<double>(n) * step < 50.0) ++n;
    const int per = (n + 63) / 64;
    const int k0 = 1 + lane * per, k1 = k0 + per - 1 < n ? k0 + per - 1 : n;
    double best = 0.0, best_r = 0.0;
    bool found = false;
    if (k0 <= k1) {
        double a = k0 == 1 ? 0.01 : 0.01 + static_cast<double>(k0 - 1) * step, Va, Da;
        delta(c, 0.0, a, &Va, &Da);
        for (int k = k0; k <= k1; ++k) {
            const double b = 0.01 + static_cast<double>(k) * step;
            double Vb, Db;
            delta(c, 0.0, b, &Vb, &Db);
            if (Da < 0.0 && Db >= 0.0) {
                double lo = a, hi = b;
                for (int it = 0; it < 200; ++it) {
                    const double m = 0.5 * (lo + hi);
                    if (m <= lo || m >= hi) break;
                    double Vm, Dm;
                    delta(c, 0.0, m, &Vm, &Dm);
                    if (Dm < 0.0) lo = m; else hi = m;
                }
                const double rm = 0.5 * (lo + hi);
                double Vm, Dm;
                delta(c, 0.0, rm, &Vm, &Dm);
                if (Vm < best) {
                    best = Vm;
                    best_r = rm;
                    found = true;
                }
            }
            a = b;
            Da = Db;
        }
    }
    // least value over the lanes, the lowest lane among equals
    double v = found ? best : INFINITY;
    int who = found ? lane : 64;
    for (int off = 32; off > 0; off >>= 1) {
        const double v2 = __shfl_xor(v, off);
        const int w2 = __shfl_xor(who, off);
        if (v2 < v || (v2 == v && w2 < who)) {
            v = v2;
            who = w2;
        }
    }
    if (who >= 64) return false;
    const double r = __shfl(best_r, who);
    *chi_e = sqrt(-v);
    *r_e = r;
    return true;
}

__global__ __launch_bounds__(256) void scan_kernel(const rt_scan_point* __restrict__ pts, int32_t n,
                                                   double* __restrict__ out) {
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
    if (i >= n) return;   // whole wavefronts
    const rt_scan_point q = pts[i];
    const double nan = __builtin_nan("");
    double res[4] = {nan, nan, nan, nan};
    const bool ok_metric = q.metric == RT_KERR ||
                           (q.metric == RT_EINASTO && q.halo[0] > 0.0) ||
                           (q.metric == RT_CNFW && q.halo[0] >= 0.0 && q.halo[1] > 0.0);
    if (ok_metric && q.reserved == 0 && isfinite(q.spin) && isfinite(q.theta) &&
        isfinite(q.halo[0]) && isfinite(q.halo[1])) {
        ImageConst c{};
        c.metric = q.metric;
        c.chi = q.spin;
        c.chi2 = q.spin * q.spin;
        if (q.metric == RT_EINASTO) c.inv_lam = 1.0 / q.halo[0];
        if (q.metric == RT_CNFW) {
            c.lam_c = q.halo[1];
            c.inv_lam_c = 1.0 / q.halo[1];
            c.eta_lc = q.halo[0] * q.halo[1];
        }
        double r;
        if (largest_root_wave(c, c.chi2, &r)) res[0] = r;
        const double co = cos(q.theta);
        if (largest_root_wave(c, c.chi2 * co * co, &r)) res[1] = r;
        double chi_e, r_e;
        if (extremal_spin_wave(c, &chi_e, &r_e)) {
            res[2] = chi_e;
            res[3] = r_e;
        }
    }
    if (__lane_id() == 0)
        for (int j = 0; j < 4; ++j) out[4 * i + j] = res[j];
}

}  // namespace

hipError_t launch_scan(const ::rt_scan_point* pts, int32_t n, double* out, hipStream_t stream) {
    const int64_t threads = static_cast<int64_t>(n) * 64;
    hipLaunchKernelGGL(scan_kernel, dim3(static_cast<uint32_t>((threads + 255) / 256)), dim3(256), 0,
                       stream, pts, n, out);
    return hipGetLastError();
}

}  // namespace rt
