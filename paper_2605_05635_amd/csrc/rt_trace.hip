// rt_trace.hip -- gfx950 kernels of the backward null-geodesic ray tracer.
//
// One wavefront lane integrates one ray (one screen pixel) from the observer
// toward the hole with Hamilton's equations (Sec. 3.1, eqs. (46)-(47) and
// (57)-(62)) and an adaptive Dormand-Prince 5(4) step controller, detects
// equatorial crossings on the step's continuous extension (Sec. 3.3, 4.2) and
// records the transfer maps of the first three crossings (Sec. 4.3, eq. (82)).
// A second, one-thread-per-pixel pass computes the redshifted thin-disc
// intensity of the recorded crossings (Sec. 5.2, eqs. (89)-(91)) and writes NaN
// into the transfer-map records beyond them.
//
// Launch shape: a persistent grid.  Each wavefront claims chunks of pixels
// from a global counter with one atomic per chunk; a lane whose ray ends takes
// the next pixel of its wave's chunk at the next refill point, so lanes stay
// busy while rays of very different lengths are in flight (wavefront-level
// compaction of terminated rays).  Two kernels share every line of per-ray
// code: trace_kernel<metric> for one image (its constants are kernel
// arguments, held in scalar registers) and trace_batch_kernel for many images
// of any metrics in one launch (their constants staged in LDS, each lane
// carrying the few its step loop needs).  Compiled with floating-point
// contraction limited to single expressions, the two produce bit-identical
// rays.
#include "rt_ray.h"

namespace rt {
namespace {

using namespace ray;

// The register allocation aims at three waves per SIMD (at most 168 VGPRs;
// the cored NFW spills three values): measured 5-10 % faster than two.
constexpr int kTraceWaves = 3;


// Persistent trace kernel for one image (pixels handed out as shape says).
template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kTraceWaves, 8))) void trace_kernel(
    ImageConst c, OutPtrs o, unsigned long long* queue, LaunchShape shape) {
    const Hot k = hot_of(c);
    Ray r;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;   // wave-uniform: claimed ordinals not yet started
    TileClaim tc{0, 0, 1, 1.0f};
    auto claim = [&]() { return claim_screen(shape, c.nx, c.ny, queue, next, end, tc); };
    auto take = [&](int64_t ordinal) {
        start_ray<METRIC>(c, k, claimed(shape, c.nx, c.ny, tc, ordinal), r);
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            const int32_t st = attempt<METRIC>(k, o, c.n_pix, r);
            if (st != 0) {
                finish_ray<false>(c, o, r, st);
                active = false;
            }
        }
    }
}

// Persistent trace kernel for a batch of images.  The images' constants are
// copied into LDS once per workgroup; the work queue enumerates chunks of all
// images (images ordered by metric, so a wavefront's lanes share a metric
// except at the two metric boundaries).  Each lane keeps its image index and
// the step-loop constants of that image in registers.  Register-allocated for
// three waves per SIMD (167 VGPRs, 21 values spilled): 5 % faster than two.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void trace_batch_kernel(
    const ImageConst* __restrict__ table, const OutPtrs* __restrict__ outs,
    const int64_t* __restrict__ chunk_start, int32_t n_images, unsigned long long* queue,
    LaunchShape shape) {
    extern __shared__ unsigned char lds_raw[];
    ImageConst* lt = reinterpret_cast<ImageConst*>(lds_raw);
    int64_t* lcs = reinterpret_cast<int64_t*>(lds_raw + sizeof(ImageConst) * n_images);
    {
        const int words = static_cast<int>(sizeof(ImageConst) / 8) * n_images;
        const uint64_t* src = reinterpret_cast<const uint64_t*>(table);
        uint64_t* dst = reinterpret_cast<uint64_t*>(lt);
        for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
        for (int i = threadIdx.x; i <= n_images; i += blockDim.x) lcs[i] = chunk_start[i];
    }
    __syncthreads();
    const int64_t total_chunks = lcs[n_images];

    Ray r;
    Hot k{};
    int32_t img = 0, metric = KERR;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    int32_t cur = 0;   // wave-uniform image of the current chunk
    auto claim = [&]() {
        unsigned long long q = 0;
        if (__lane_id() == 0) q = atomicAdd(queue, 1ull);
        q = __shfl(q, 0);
        if (static_cast<int64_t>(q) >= total_chunks) return false;
        // image of chunk q: the last i with chunk_start[i] <= q
        int32_t lo = 0, hi = n_images - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (lcs[mid] <= static_cast<int64_t>(q)) lo = mid; else hi = mid - 1;
        }
        cur = lo;
        const int64_t npix = lt[cur].n_pix;
        next = (static_cast<int64_t>(q) - lcs[cur]) * shape.chunk;
        end = next + shape.chunk < npix ? next + shape.chunk : npix;
        return true;
    };
    auto take = [&](int64_t ordinal) {
        img = cur;
        const ImageConst& c = lt[img];
        metric = (c.metric == CNFW && c.ex_near) ? CNFW_NEAR : c.metric;
        k = hot_of(c);
        // (the pixel's row and column by quotient(): no integer division)
        Pixel px;
        px.pix = tile_pixel(ordinal, c.nx, c.ny, shape.tile_w, shape.tile_h, FpQuotient{});
        px.iy = quotient(static_cast<int32_t>(px.pix), c.nx);
        px.ix = static_cast<int32_t>(px.pix) - px.iy * c.nx;
        if (metric == CNFW_NEAR) start_ray<CNFW_NEAR>(c, k, px, r);
        else if (metric == CNFW) start_ray<CNFW>(c, k, px, r);
        else if (metric == EINASTO) start_ray<EINASTO>(c, k, px, r);
        else start_ray<KERR>(c, k, px, r);
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            const OutPtrs& o = outs[img];
            const int64_t n_pix = lt[img].n_pix;
            int32_t st;
            if (metric == CNFW_NEAR) st = attempt<CNFW_NEAR>(k, o, n_pix, r);
            else if (metric == CNFW) st = attempt<CNFW>(k, o, n_pix, r);
            else if (metric == EINASTO) st = attempt<EINASTO>(k, o, n_pix, r);
            else st = attempt<KERR>(k, o, n_pix, r);
            if (st != 0) {
                finish_ray<false>(lt[img], o, r, st);
                active = false;
            }
        }
    }
}

// Emission pass of one image, one thread per pixel, after its trace.
template <int METRIC>
__global__ __launch_bounds__(kBlock) void emission_kernel(ImageConst c, OutPtrs o) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p < c.n_pix) emit_pixel<METRIC>(c, hot_of(c), o, p);
}

// Emission pass of a batch of images: image blockIdx.y, pixels by blockIdx.x.
__global__ __launch_bounds__(kBlock) void emission_batch_kernel(
    const ImageConst* __restrict__ table, const OutPtrs* __restrict__ outs) {
    const ImageConst c = table[blockIdx.y];
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= c.n_pix) return;
    const OutPtrs o = outs[blockIdx.y];
    const Hot k = hot_of(c);
    if (c.metric == CNFW)
        emit_pixel<CNFW>(c, k, o, p);
    else if (c.metric == EINASTO)
        emit_pixel<EINASTO>(c, k, o, p);
    else
        emit_pixel<KERR>(c, k, o, p);
}

__global__ void zero_counters(unsigned long long* q, int32_t n) {
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) q[i] = 0ull;
}

}  // namespace

hipError_t launch_zero(unsigned long long* queue, int32_t n, hipStream_t stream) {
    hipLaunchKernelGGL(zero_counters, dim3((n + 255) / 256), dim3(256), 0, stream, queue, n);
    return hipGetLastError();
}

hipError_t launch_trace(const ImageConst& c, const OutPtrs& o, unsigned long long* queue,
                        const LaunchShape& shape, int32_t grid, hipStream_t stream) {
    switch (c.metric) {
        case KERR:
            hipLaunchKernelGGL(trace_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                               queue, shape);
            break;
        case EINASTO:
            hipLaunchKernelGGL(trace_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                               queue, shape);
            break;
        default:
            if (c.ex_near)
                hipLaunchKernelGGL(trace_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream, c,
                                   o, queue, shape);
            else
                hipLaunchKernelGGL(trace_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c, o,
                                   queue, shape);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_emission(const ImageConst& c, const OutPtrs& o, hipStream_t stream) {
    const dim3 grid(static_cast<unsigned>((c.n_pix + kBlock - 1) / kBlock));
    switch (c.metric) {
        case KERR:
            hipLaunchKernelGGL(emission_kernel<KERR>, grid, dim3(kBlock), 0, stream, c, o);
            break;
        case EINASTO:
            hipLaunchKernelGGL(emission_kernel<EINASTO>, grid, dim3(kBlock), 0, stream, c, o);
            break;
        default:
            hipLaunchKernelGGL(emission_kernel<CNFW>, grid, dim3(kBlock), 0, stream, c, o);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_emission_batch(const ImageConst* table, const OutPtrs* outs, int32_t n_images,
                                 int64_t max_pix, hipStream_t stream) {
    const dim3 grid(static_cast<unsigned>((max_pix + kBlock - 1) / kBlock),
                    static_cast<unsigned>(n_images));
    hipLaunchKernelGGL(emission_batch_kernel, grid, dim3(kBlock), 0, stream, table, outs);
    return hipGetLastError();
}

size_t batch_lds_bytes(int32_t n_images) {
    return sizeof(ImageConst) * static_cast<size_t>(n_images) +
           sizeof(int64_t) * static_cast<size_t>(n_images + 1);
}

hipError_t launch_trace_batch(const ImageConst* table, const OutPtrs* outs,
                              const int64_t* chunk_start, int32_t n_images,
                              unsigned long long* queue, const LaunchShape& shape, int32_t grid,
                              hipStream_t stream) {
    hipLaunchKernelGGL(trace_batch_kernel, dim3(grid), dim3(kBlock), batch_lds_bytes(n_images),
                       stream, table, outs, chunk_start, n_images, queue, shape);
    return hipGetLastError();
}

int max_blocks_per_cu(int metric) {
    int n = 0;
    hipError_t e;
    if (metric == KERR)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, trace_kernel<KERR>, kBlock, 0);
    else if (metric == EINASTO)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, trace_kernel<EINASTO>, kBlock, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, trace_kernel<CNFW>, kBlock, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

int max_batch_blocks_per_cu(int32_t n_images) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, trace_batch_kernel, kBlock, batch_lds_bytes(n_images));
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace rt
