// rt_boundary.hip -- gfx950 kernel of the shadow-boundary search (Sec. 4.1,
// eqs. (78)-(79)): along a screen direction (cos psi, sin psi), the impact
// parameter b at which the rays from X = b cos psi, Y = b sin psi turn from
// captured to escaping.  A wavefront holds 64 / S directions, S lanes each
// (S = 64, 32 or 16 samples per pass); each pass traces one ray per lane at
// the S interior points of its direction's bracket and keeps the interval
// around the first escaping one, so the bracket shrinks (S + 1)-fold per pass
// instead of 2-fold per traced ray.  The directions of a wavefront advance
// independently, each from pass to pass as soon as its own rays end.  Fewer samples per direction trace fewer
// rays in all and put more directions in flight; more samples need fewer
// passes.
#include "rt_ray.h"

namespace rt {
namespace {

using namespace ray;

constexpr int kMaxPasses = 64;

// Register-allocated like the trace kernel (three waves per SIMD).
template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void boundary_kernel(
    ImageConst c, const double* __restrict__ dirs, int32_t n, int32_t S, double b_lo, double b_hi,
    double b_tol, double* __restrict__ out, int32_t* __restrict__ status,
    int64_t* __restrict__ attempts) {
    const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / 64;
    const int lane = __lane_id();
    const int G = 64 / S;                    // directions per wavefront
    const int grp = lane / S, sl = lane - grp * S;
    const int64_t dir = wave * G + grp;
    const unsigned long long gmask = S == 64 ? ~0ull : ((1ull << S) - 1ull);
    const Hot k = hot_of(c);
    const OutPtrs none{};    // no per-pixel outputs
    const bool mine = dir < n;
    const double ux = mine ? dirs[2 * dir] : 0.0, uy = mine ? dirs[2 * dir + 1] : 0.0;
    double lo = b_lo, hi = b_hi;
    int64_t used = 0;        // this lane's step attempts
    int32_t result = 1;      // bracket without the transition, until checked
    bool done = !mine;
    // Pass -1 checks the bracket (sample 0 at b_lo must stay inside, sample 1
    // at b_hi must escape); passes 0, 1, ... sample b_j = lo + j w, j = sl + 1.
    // Each group runs its passes on its own: when the last of its rays ends it
    // narrows its bracket and starts its next pass at once, while the other
    // groups' rays are still in flight (a pass no longer waits for the
    // slowest ray of the whole wavefront).
    int pass = -1;
    Ray r;
    bool active = false;     // this lane's ray is in flight
    bool escaped = false;    // the fate of its ray in the group's current pass
    auto start_pass = [&]() {
        const double w = (hi - lo) / (S + 1);
        double b;
        if (pass < 0) {
            b = sl == 0 ? b_lo : b_hi;
        } else {
            const double t = static_cast<double>(sl + 1) * w;   // no contraction
            b = lo + t;
        }
        active = pass >= 0 || sl < 2;
        escaped = false;
        if (active) start_ray_dir<METRIC>(c, k, screen_dir_xy(c, b * ux, b * uy), 0, r);
    };
    if (!done) start_pass();
    while (__ballot(!done) != 0ull) {
        if (active) {
            const int32_t st = attempt<METRIC>(k, none, 0, r);
            if (st != 0) {
                active = false;
                escaped = st == RAY_ESCAPED;
                used += r.attempts;
            }
        }
        const unsigned long long busy = (__ballot(active) >> (grp * S)) & gmask;
        const unsigned long long esc = (__ballot(escaped) >> (grp * S)) & gmask;
        if (!done && busy == 0ull) {
            // the group's pass is complete: the same bracket update as a
            // lockstep search would make
            if (pass < 0) {
                if ((esc & 1ull) || !(esc & 2ull)) {
                    done = true;
                } else {
                    result = 0;
                }
            } else {
                const double w = (hi - lo) / (S + 1);
                double nlo, nhi;
                if (esc == 0ull) {
                    const double t = S * w;
                    nlo = lo + t;
                    nhi = hi;
                } else {
                    const int j = __ffsll(static_cast<long long>(esc));   // first escaping sample
                    const double tj = j * w, tj1 = (j - 1) * w;
                    nhi = lo + tj;
                    nlo = j == 1 ? lo : lo + tj1;
                }
                if (nlo == lo && nhi == hi) {
                    done = true;   // below the resolution of b
                } else {
                    lo = nlo;
                    hi = nhi;
                }
            }
            if (pass + 1 >= kMaxPasses || !(hi - lo > b_tol)) done = true;
            ++pass;
            if (!done) start_pass();
        }
    }
    // the group's attempt total, in a fixed order
    for (int off = S / 2; off > 0; off >>= 1) used += __shfl_xor(used, off);
    if (mine && sl == 0) {
        out[2 * dir] = lo;
        out[2 * dir + 1] = hi;
        status[dir] = result;
        if (attempts) attempts[dir] = used;
    }
}

}  // namespace

hipError_t launch_boundary(const ImageConst& c, const double* dirs, int32_t n, int32_t samples,
                           double b_lo, double b_hi, double b_tol, double* out, int32_t* status,
                           int64_t* attempts, hipStream_t stream) {
    const int64_t waves = (static_cast<int64_t>(n) * samples + 63) / 64;
    const int32_t blocks = static_cast<int32_t>((waves + kBlock / 64 - 1) / (kBlock / 64));
    if (c.metric == KERR)
        hipLaunchKernelGGL(boundary_kernel<KERR>, dim3(blocks), dim3(kBlock), 0, stream, c, dirs,
                           n, samples, b_lo, b_hi, b_tol, out, status, attempts);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(boundary_kernel<EINASTO>, dim3(blocks), dim3(kBlock), 0, stream, c,
                           dirs, n, samples, b_lo, b_hi, b_tol, out, status, attempts);
    else if (c.ex_near)
        hipLaunchKernelGGL(boundary_kernel<CNFW_NEAR>, dim3(blocks), dim3(kBlock), 0, stream, c,
                           dirs, n, samples, b_lo, b_hi, b_tol, out, status, attempts);
    else
        hipLaunchKernelGGL(boundary_kernel<CNFW>, dim3(blocks), dim3(kBlock), 0, stream, c, dirs,
                           n, samples, b_lo, b_hi, b_tol, out, status, attempts);
    return hipGetLastError();
}

}  // namespace rt
