// rt_scan.hip -- parameter scans of the spacetimes (Sec. 2): per point, the
// outer horizon (eq. (33)), the ergosurface radius at one polar angle, and the
// extremal spin with its radius, one thread per point (rt_scan.h).
#include "rt.h"
#include "rt_scan.h"

namespace rt {
namespace {

__global__ __launch_bounds__(256) void scan_kernel(const rt_scan_point* __restrict__ pts, int32_t n,
                                                   double* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
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
        if (scan::largest_root(c, c.chi2, &r)) res[0] = r;
        const double co = cos(q.theta);
        if (scan::largest_root(c, c.chi2 * co * co, &r)) res[1] = r;
        double chi_e, r_e;
        if (scan::extremal_spin(c, &chi_e, &r_e)) {
            res[2] = chi_e;
            res[3] = r_e;
        }
    }
    for (int j = 0; j < 4; ++j) out[4 * i + j] = res[j];
}

}  // namespace

hipError_t launch_scan(const ::rt_scan_point* pts, int32_t n, double* out, hipStream_t stream) {
    hipLaunchKernelGGL(scan_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, pts, n, out);
    return hipGetLastError();
}

}  // namespace rt
