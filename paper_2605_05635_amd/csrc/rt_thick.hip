// rt_thick.hip -- gfx950 kernel of the thick-disc image (Sec. 5.1-5.2): the
// persistent trace of rt_trace.hip with the intensity I = int g^3 j dlambda
// as a seventh, error-controlled Dormand-Prince component (attempt<..., THICK>).
#include "rt_ray.h"

namespace rt {
namespace {

using namespace ray;

// The image's constants reloaded from the kernel-argument segment (scalar
// loads through the scalar cache) where they are used, instead of held in
// scalar registers across the step loop: the thick attempt needs those
// registers for its own constants (held, ~90 scalar registers spilled into
// vector-register lanes, a tenth of its vector instructions reading them
// back).  The empty asm hides the pointer's value from the compiler, so the
// loads stay where they are written.  `c`, the kernel's first argument, sits
// at the segment's start.
__device__ __forceinline__ const ImageConst& reloaded_args() {
    const ImageConst* q = (const ImageConst*)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(q));
    return *q;
}

template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void trace_thick_kernel(
    ImageConst c, OutPtrs o, unsigned long long* queue, LaunchShape shape) {
    Ray r;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    TileClaim tc{0, 0, 1, 1.0f};
    auto claim = [&]() {
        const ImageConst& a = reloaded_args();
        return claim_screen(shape, a.nx, a.ny, queue, next, end, tc);
    };
    auto take = [&](int64_t ordinal) {
        const ImageConst& a = reloaded_args();
        start_ray_thick<METRIC>(a, hot_of(a), claimed_pixel(shape, a.nx, a.ny, tc, ordinal), r);
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            const int32_t st = attempt<METRIC, StageNone, true>(hot_of(reloaded_args()), o, c.n_pix, r);
            if (st != 0) {
                finish_ray(reloaded_args(), o, r, st);
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
