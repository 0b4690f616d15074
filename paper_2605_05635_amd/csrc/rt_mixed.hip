// rt_mixed.hip -- gfx950 kernels of the mixed-precision trace: a persistent
// binary32 pass over the screen (rt_ray32.h) that finishes most rays and hands
// the others to a list (rays entering the horizon zone with their state, rays
// to trace again with their pixel), then a persistent binary64 pass over that
// list.  The list length stays on the device: the second kernel reads it, so
// the two launches need no host round trip.
#include "rt_ray32.h"

namespace rt {
namespace {

using namespace ray;
using namespace ray32;

// Adds the wave's sum of v to *total (one atomic per wave, from lane 0).
// Called by every lane of the wave, converged.
__device__ __forceinline__ void add_wave_total(uint32_t v, unsigned long long* total) {
    unsigned long long s = v;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (__lane_id() == 0) atomicAdd(total, s);
}

// Register-allocated for four waves per SIMD (128 VGPRs, a few spilled):
// measured 6 % faster than three.
template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void trace32_kernel(ImageConst c, OutPtrs o,
                                                         unsigned long long* queue,
                                                         LaunchShape shape, double* records,
                                                         unsigned int* counters) {
    const Hot32 k = hot32_of(c);
    Ray32 r;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    TileClaim tc{0, 0, 1, 1.0f};
    auto claim = [&]() { return claim_screen(shape, c.nx, c.ny, queue, next, end, tc); };
    auto take = [&](int64_t ordinal) {
        start_ray32<METRIC>(c, k, claimed_pixel(shape, c.nx, c.ny, tc, ordinal), r);
    };
    const int lane = __lane_id();
    uint32_t tried = 0;   // this lane's binary32 step attempts
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        int32_t leave = 0;
        if (active) {
            ++tried;
            const int32_t st = attempt32<METRIC>(k, o, c.n_pix, r);
            if (st > 0) {
                Ray w;
                widen(c, r, w);
                finish_ray(c, o, w, st);
                active = false;
            } else if (st < 0) {
                leave = st;
                active = false;
            }
        }
        // Rays leaving binary32 append a record to the list: one atomic per wave.
        const unsigned long long m = __ballot(leave != 0);
        if (m != 0ull) {
            const unsigned long long mr = __ballot(leave == kRerun);
            const int leader = __ffsll(static_cast<long long>(m)) - 1;
            unsigned int base = 0;
            if (lane == leader) {
                base = atomicAdd(&counters[0], static_cast<unsigned int>(__popcll(m)));
                if (mr != 0ull) atomicAdd(&counters[1], static_cast<unsigned int>(__popcll(mr)));
            }
            base = __shfl(base, leader);
            if (leave != 0) {
                const unsigned int slot = base + __popcll(m & ((1ull << lane) - 1ull));
                double* rec = records + static_cast<int64_t>(slot) * kRecord;
                if (leave == kHandOff) {
                    Ray w;
                    widen(c, r, w);
                    store_record(rec, w);
                } else {
                    store_rerun(rec, r.pix);
                }
            }
        }
    }
    add_wave_total(tried, reinterpret_cast<unsigned long long*>(counters + 4));
}

// A continued ray that reaches its second crossing is traced again from the
// screen as well (and counted in counters[1]), so that every ray with two
// crossings has its binary64 outputs.  Register-allocated for three waves per
// SIMD, as the binary64 trace kernel: the pass is short (a third of the rays)
// and ends on its longest rays, so it needs every wave it can keep resident.
template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void resume_kernel(
    ImageConst c, OutPtrs o, const double* __restrict__ records, unsigned int* counters,
    unsigned long long* queue, int32_t chunk) {
    const Hot k = hot_of(c);
    const int64_t total = counters[0];
    Ray r;
    bool fresh = false;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    auto claim = [&]() { return claim_chunk(queue, chunk, total, next, end); };
    auto take = [&](int64_t e) {
        const double* rec = records + e * kRecord;
        load_record<METRIC>(c, k, rec, r);
        fresh = rec[18] != 0.0;
    };
    uint32_t tried = 0;   // this lane's binary64 step attempts
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            ++tried;
            const int32_t st = attempt<METRIC>(k, o, c.n_pix, r);
            if (!fresh && r.ncross >= kRerunCrossings) {
                start_ray<METRIC>(c, k, r.pix, r);
                fresh = true;
                atomicAdd(&counters[1], 1u);
            } else if (st != 0) {
                finish_ray(c, o, r, st);
                active = false;
            }
        }
    }
    add_wave_total(tried, reinterpret_cast<unsigned long long*>(counters + 6));
}

__global__ void copy_counters(const unsigned int* __restrict__ counters,
                              long long* __restrict__ stats) {
    const unsigned long long* wide = reinterpret_cast<const unsigned long long*>(counters + 4);
    if (threadIdx.x < 2) stats[threadIdx.x] = static_cast<long long>(counters[threadIdx.x]);
    if (threadIdx.x >= 2 && threadIdx.x < 4)
        stats[threadIdx.x] = static_cast<long long>(wide[threadIdx.x - 2]);
}

template <class Kern>
int occupancy(Kern kern) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBlock, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

size_t mixed_record_bytes() { return sizeof(double) * kRecord; }

hipError_t launch_trace32(const ImageConst& c, const OutPtrs& o, unsigned long long* queue,
                          const LaunchShape& shape, int32_t grid, double* records,
                          unsigned int* counters, hipStream_t stream) {
    if (c.metric == KERR)
        hipLaunchKernelGGL(trace32_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c, o, queue,
                           shape, records, counters);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(trace32_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                           queue, shape, records, counters);
    else if (c.ex_near)
        hipLaunchKernelGGL(trace32_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                           queue, shape, records, counters);
    else
        hipLaunchKernelGGL(trace32_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c, o, queue,
                           shape, records, counters);
    return hipGetLastError();
}

hipError_t launch_resume(const ImageConst& c, const OutPtrs& o, const double* records,
                         unsigned int* counters, unsigned long long* queue, int32_t chunk,
                         int32_t grid, hipStream_t stream) {
    if (c.metric == KERR)
        hipLaunchKernelGGL(resume_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c, o, records,
                           counters, queue, chunk);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(resume_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                           records, counters, queue, chunk);
    else if (c.ex_near)
        hipLaunchKernelGGL(resume_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                           records, counters, queue, chunk);
    else
        hipLaunchKernelGGL(resume_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c, o, records,
                           counters, queue, chunk);
    return hipGetLastError();
}

hipError_t launch_copy_counters(const unsigned int* counters, long long* stats,
                                hipStream_t stream) {
    hipLaunchKernelGGL(copy_counters, dim3(1), dim3(64), 0, stream, counters, stats);
    return hipGetLastError();
}

int mixed_blocks_per_cu(int metric, int pass) {
    if (pass == 0) {
        if (metric == KERR) return occupancy(trace32_kernel<KERR>);
        if (metric == EINASTO) return occupancy(trace32_kernel<EINASTO>);
        return occupancy(trace32_kernel<CNFW>);
    }
    if (metric == KERR) return occupancy(resume_kernel<KERR>);
    if (metric == EINASTO) return occupancy(resume_kernel<EINASTO>);
    return occupancy(resume_kernel<CNFW>);
}

}  // namespace rt
