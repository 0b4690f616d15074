// rt_points.hip -- gfx950 kernels of the adaptive screen: rays traced from a
// list of screen points, and the refinement of a traced screen near its
// lensing-band boundaries.  The paper resolves the shadow boundary, the
// critical curve and the higher-order images by refining the observer screen
// where the image-plane classification changes (Sec. 4, with the bands of
// Sec. 4.2 labelled by N_cross): a pixel whose 4-neighbour has another
// crossing count or another fate (captured, escaped) straddles such a change,
// and its subpixels are traced again.
#include "rt_points.h"
#include "rt_ray.h"

namespace rt {
namespace {

using namespace ray;

constexpr int32_t kPointChunk = 64;   // points per work-queue claim (one wavefront's refill)

// Persistent trace of listed points: the loop of the image trace, ray i
// starting from (X_i, Y_i) and recorded as "pixel" i; its epilogue writes the
// NaN records past min(N_cross, 3) (no pass after it but the emission).
template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void trace_points_kernel(
    ImageConst c, const double* __restrict__ xy, OutPtrs o, unsigned long long* queue) {
    const Hot k = hot_of(c);
    Ray r;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    auto claim = [&]() { return claim_chunk(queue, kPointChunk, c.n_pix, next, end); };
    auto take = [&](int64_t i) {
        start_ray_dir<METRIC>(c, k, screen_dir_xy(c, xy[2 * i], xy[2 * i + 1]), i, r);
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            const int32_t st = attempt<METRIC>(k, o, c.n_pix, r);
            if (st != 0) {
                finish_ray<true>(c, o, r, st);
                active = false;
            }
        }
    }
}

// Emission (Sec. 5.2) of point p's recorded crossings, as the image's
// per-pixel pass computes it for a pixel centre: g_n, I_n = w g_n^3 R_n^-p for
// n < min(N_cross, 3) (NaN beyond), I their sum.
template <int METRIC>
__global__ __launch_bounds__(kBlock) void emit_points_kernel(ImageConst c, const double* __restrict__ xy,
                                                             OutPtrs o) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= c.n_pix) return;
    const Hot k = hot_of(c);
    const int ncr = o.ncross[p];
    const int nrec = ncr < 3 ? ncr : 3;
    double E, L;
    photon_constants(c, screen_dir_xy(c, xy[2 * p], xy[2 * p + 1]), E, L);
    double intensity = 0.0;
    for (int n = 0; n < 3; ++n) {
        const int64_t off = static_cast<int64_t>(n) * c.n_pix + p;
        double g = __builtin_nan(""), In = __builtin_nan("");
        if (n < nrec) {
            const double R = o.r_em[off];
            g = redshift<METRIC>(k, R, E, L);
            In = disc_window(c, R, c.r_in) * g * g * g * pow(R, -c.emis_pow);
            intensity += In;
        }
        if (o.g_em) o.g_em[off] = g;
        if (o.intensity_n) o.intensity_n[off] = In;
    }
    if (o.intensity) o.intensity[p] = intensity;
}

// Whether pixel p of the nx x ny screen has a 4-neighbour with another
// crossing count or status.
__device__ __forceinline__ bool on_band_edge(const uint8_t* __restrict__ nc,
                                             const uint8_t* __restrict__ st, int32_t nx,
                                             int32_t ny, int32_t p) {
    const int32_t iy = p / nx, ix = p - iy * nx;
    const uint8_t a = nc[p], s = st[p];
    bool edge = false;
    if (ix > 0) edge |= nc[p - 1] != a || st[p - 1] != s;
    if (ix + 1 < nx) edge |= nc[p + 1] != a || st[p + 1] != s;
    if (iy > 0) edge |= nc[p - nx] != a || st[p - nx] != s;
    if (iy + 1 < ny) edge |= nc[p + nx] != a || st[p + nx] != s;
    return edge;
}

// Pass 1: marked pixels per workgroup of kBlock consecutive pixels.
__global__ __launch_bounds__(kBlock) void refine_count(ImageConst c, const uint8_t* __restrict__ nc,
                                                       const uint8_t* __restrict__ st,
                                                       int64_t* __restrict__ block_count) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool m = p < c.n_pix && on_band_edge(nc, st, c.nx, c.ny, static_cast<int32_t>(p));
    const int n = __syncthreads_count(m);
    if (threadIdx.x == 0) block_count[blockIdx.x] = n;
}

// Pass 2 (one workgroup): exclusive prefix sums of the counts in place, the
// total to *n_marked.  Each tile of kBlock counts: an inclusive scan within
// each wavefront by lane shifts, then the wavefronts' totals in order.
__global__ __launch_bounds__(kBlock) void refine_scan(int64_t* __restrict__ block_count,
                                                      int64_t n_blocks, int64_t* __restrict__ n_marked) {
    __shared__ long long wave_total[kBlock / 64];
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    long long carry = 0;
    for (int64_t base = 0; base < n_blocks; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        const long long v = i < n_blocks ? block_count[i] : 0;
        long long x = v;
        for (int d = 1; d < 64; d <<= 1) {
            const long long y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (lane == 63) wave_total[wave] = x;
        __syncthreads();
        long long before = carry, tile = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            if (w < wave) before += wave_total[w];
            tile += wave_total[w];
        }
        if (i < n_blocks) block_count[i] = before + x - v;
        carry += tile;
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_marked = carry;
}

// Pass 3: each marked pixel's rank in pixel order, its index and its
// subpixel centres.
__global__ __launch_bounds__(kBlock) void refine_scatter(ImageConst c, const uint8_t* __restrict__ nc,
                                                         const uint8_t* __restrict__ st,
                                                         const int64_t* __restrict__ block_start,
                                                         int32_t sub, int64_t max_marked,
                                                         double* __restrict__ xy,
                                                         int64_t* __restrict__ pix) {
    __shared__ int32_t wave_count[kBlock / 64];
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool m = p < c.n_pix && on_band_edge(nc, st, c.nx, c.ny, static_cast<int32_t>(p));
    const unsigned long long b = __ballot(m);
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    if (lane == 0) wave_count[wave] = __popcll(b);
    __syncthreads();
    if (!m) return;
    int64_t rank = block_start[blockIdx.x] + __popcll(b & ((1ull << lane) - 1ull));
    for (int w = 0; w < wave; ++w) rank += wave_count[w];
    if (rank >= max_marked) return;
    if (pix) pix[rank] = p;
    const int32_t iy = static_cast<int32_t>(p) / c.nx, ix = static_cast<int32_t>(p) - iy * c.nx;
    const double inv_sub = 1.0 / static_cast<double>(sub);
    double* out = xy + 2 * rank * static_cast<int64_t>(sub) * sub;
    for (int32_t bb = 0; bb < sub; ++bb) {
        const double v = (static_cast<double>(bb) + 0.5) * inv_sub;
        const double Y = c.y0 + (static_cast<double>(iy) + v) * c.dy;
        for (int32_t a = 0; a < sub; ++a) {
            const double u = (static_cast<double>(a) + 0.5) * inv_sub;
            out[0] = c.x0 + (static_cast<double>(ix) + u) * c.dx;
            out[1] = Y;
            out += 2;
        }
    }
}

template <class Kern>
int occupancy(Kern kern) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBlock, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

template <int METRIC>
hipError_t launch_points(const ImageConst& c, const double* xy, const OutPtrs& o,
                         unsigned long long* queue, int32_t grid, hipStream_t stream) {
    hipLaunchKernelGGL(trace_points_kernel<METRIC>, dim3(grid), dim3(kBlock), 0, stream, c, xy, o,
                       queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !c.emission) return e;
    const int64_t blocks = (c.n_pix + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(emit_points_kernel<METRIC>, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0,
                       stream, c, xy, o);
    return hipGetLastError();
}

}  // namespace

int points_blocks_per_cu(int metric) {
    if (metric == KERR) return occupancy(trace_points_kernel<KERR>);
    if (metric == EINASTO) return occupancy(trace_points_kernel<EINASTO>);
    return occupancy(trace_points_kernel<CNFW>);
}

hipError_t launch_trace_points(const ImageConst& c, const double* xy, const OutPtrs& o,
                               unsigned long long* queue, int32_t grid, hipStream_t stream) {
    if (c.metric == KERR) return launch_points<KERR>(c, xy, o, queue, grid, stream);
    if (c.metric == EINASTO) return launch_points<EINASTO>(c, xy, o, queue, grid, stream);
    if (c.ex_near) return launch_points<CNFW_NEAR>(c, xy, o, queue, grid, stream);
    return launch_points<CNFW>(c, xy, o, queue, grid, stream);
}

hipError_t launch_refine(const ImageConst& c, const uint8_t* ncross, const uint8_t* status,
                         int32_t sub, int64_t max_marked, double* xy, int64_t* pix,
                         int64_t* n_marked, int64_t* block_count, hipStream_t stream) {
    const int64_t blocks = (c.n_pix + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(refine_count, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, stream, c,
                       ncross, status, block_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(refine_scan, dim3(1), dim3(kBlock), 0, stream, block_count, blocks, n_marked);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(refine_scatter, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, stream, c,
                       ncross, status, block_count, sub, max_marked, xy, pix);
    return hipGetLastError();
}

}  // namespace rt
