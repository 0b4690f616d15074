// rt_boundary.hip -- gfx950 kernel of the shadow-boundary search (Sec. 4.1,
// eqs. (78)-(79)): along a screen direction (cos psi, sin psi), the impact
// parameter b at which the rays from X = b cos psi, Y = b sin psi turn from
// captured to escaping.  One wavefront per direction; each pass traces one
// ray per lane at 64 points inside the bracket and keeps the interval around
// the first escaping one, so the bracket shrinks 65-fold per pass (7 passes
// from a width of 10 to 1e-12) instead of 2-fold per traced ray.
#include "rt_ray.h"

namespace rt {
namespace {

using namespace ray;

constexpr int kSamples = 64;     // rays per pass: one per lane of a wavefront
constexpr int kMaxPasses = 64;

// Register-allocated like the trace kernel (three waves per SIMD).
template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void boundary_kernel(
    ImageConst c, const double* __restrict__ dirs, int32_t n, double b_lo, double b_hi,
    double b_tol, double* __restrict__ out, int32_t* __restrict__ status,
    int64_t* __restrict__ attempts) {
    const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / 64;
    if (wave >= n) return;   // whole wavefronts: kBlock is a multiple of 64
    const int lane = __lane_id();
    const Hot k = hot_of(c);
    const OutPtrs none{};    // no per-pixel outputs
    const double ux = dirs[2 * wave], uy = dirs[2 * wave + 1];
    double lo = b_lo, hi = b_hi;
    int64_t used = 0;        // this lane's step attempts
    int32_t result = 1;      // bracket without the transition, until checked
    // Pass -1 checks the bracket (lane 0 at b_lo must stay inside, lane 1 at
    // b_hi must escape); passes 0, 1, ... sample b_j = lo + j w, j = lane + 1.
    for (int pass = -1;; ++pass) {
        const double w = (hi - lo) / (kSamples + 1);
        double b;
        if (pass < 0) {
            b = lane == 0 ? b_lo : b_hi;
        } else {
            const double t = static_cast<double>(lane + 1) * w;   // no contraction
            b = lo + t;
        }
        const bool live = pass >= 0 || lane < 2;
        Ray r;
        bool active = live;
        int32_t st = 0;
        if (live) start_ray_dir<METRIC>(c, k, screen_dir_xy(c, b * ux, b * uy), 0, r);
        while (__ballot(active) != 0ull) {
            if (active) {
                st = attempt<METRIC>(k, none, 0, r);
                if (st != 0) active = false;
            }
        }
        if (live) used += r.attempts;
        const unsigned long long esc = __ballot(live && st == RAY_ESCAPED);
        if (pass < 0) {
            if ((esc & 1ull) || !(esc & 2ull)) break;
            result = 0;
        } else {
            double nlo, nhi;
            if (esc == 0ull) {
                const double t = kSamples * w;
                nlo = lo + t;
                nhi = hi;
            } else {
                const int j = __ffsll(static_cast<long long>(esc));   // first escaping sample
                const double tj = j * w, tj1 = (j - 1) * w;
                nhi = lo + tj;
                nlo = j == 1 ? lo : lo + tj1;
            }
            if (nlo == lo && nhi == hi) break;   // below the resolution of b
            lo = nlo;
            hi = nhi;
        }
        if (pass + 1 >= kMaxPasses || !(hi - lo > b_tol)) break;
    }
    for (int off = 32; off > 0; off >>= 1) used += __shfl_xor(used, off);
    if (lane == 0) {
        out[2 * wave] = lo;
        out[2 * wave + 1] = hi;
        status[wave] = result;
        if (attempts) attempts[wave] = used;
    }
}

}  // namespace

hipError_t launch_boundary(const ImageConst& c, const double* dirs, int32_t n, double b_lo,
                           double b_hi, double b_tol, double* out, int32_t* status,
                           int64_t* attempts, hipStream_t stream) {
    const int32_t blocks = (n + kBlock / 64 - 1) / (kBlock / 64);
    if (c.metric == KERR)
        hipLaunchKernelGGL(boundary_kernel<KERR>, dim3(blocks), dim3(kBlock), 0, stream, c, dirs,
                           n, b_lo, b_hi, b_tol, out, status, attempts);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(boundary_kernel<EINASTO>, dim3(blocks), dim3(kBlock), 0, stream, c,
                           dirs, n, b_lo, b_hi, b_tol, out, status, attempts);
    else if (c.ex_near)
        hipLaunchKernelGGL(boundary_kernel<CNFW_NEAR>, dim3(blocks), dim3(kBlock), 0, stream, c,
                           dirs, n, b_lo, b_hi, b_tol, out, status, attempts);
    else
        hipLaunchKernelGGL(boundary_kernel<CNFW>, dim3(blocks), dim3(kBlock), 0, stream, c, dirs,
                           n, b_lo, b_hi, b_tol, out, status, attempts);
    return hipGetLastError();
}

}  // namespace rt
