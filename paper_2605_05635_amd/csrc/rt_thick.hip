// rt_thick.hip -- gfx950 kernel of the thick-disc image (Sec. 5.1-5.2): the
// persistent trace of rt_trace.hip with the intensity I = int g^3 j dlambda
// as a seventh, error-controlled Dormand-Prince component (attempt<..., THICK>).
#include "rt_ray.h"

namespace rt {
namespace {

using namespace ray;

template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void trace_thick_kernel(
    ImageConst c, OutPtrs o, unsigned long long* queue, LaunchShape shape) {
    const Hot k = hot_of(c);
    Ray r;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    TileClaim tc{0, 0, 1, 1.0f};
    auto claim = [&]() { return claim_screen(shape, c.nx, c.ny, queue, next, end, tc); };
    auto take = [&](int64_t ordinal) {
        start_ray_thick<METRIC>(c, k, claimed_pixel(shape, c.nx, c.ny, tc, ordinal), r);
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            const int32_t st = attempt<METRIC, StageNone, true>(k, o, c.n_pix, r);
            if (st != 0) {
                finish_ray(c, o, r, st);
                o.intensity[r.pix] = r.I;
                active = false;
            }
        }
    }
}

template <class Kern>
int occupancy(Kern kern) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBlock, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

int thick_blocks_per_cu(int metric) {
    if (metric == KERR) return occupancy(trace_thick_kernel<KERR>);
    if (metric == EINASTO) return occupancy(trace_thick_kernel<EINASTO>);
    return occupancy(trace_thick_kernel<CNFW>);
}

hipError_t launch_trace_thick(const ImageConst& c, const OutPtrs& o, unsigned long long* queue,
                              const LaunchShape& shape, int32_t grid, hipStream_t stream) {
    if (c.metric == KERR)
        hipLaunchKernelGGL(trace_thick_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                           queue, shape);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(trace_thick_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                           queue, shape);
    else if (c.ex_near)
        hipLaunchKernelGGL(trace_thick_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                           queue, shape);
    else
        hipLaunchKernelGGL(trace_thick_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                           queue, shape);
    return hipGetLastError();
}

}  // namespace rt
