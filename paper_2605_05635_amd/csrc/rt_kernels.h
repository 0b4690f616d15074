// rt_kernels.h -- host-visible launch interface of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rt_device.h"

namespace rt {

constexpr int kBlock = 256;  // 4 wavefronts of 64 lanes

// Device output pointers of one image (any may be null).
struct OutPtrs {
    uint8_t* ncross;
    uint8_t* status;
    double* r_em;
    double* phi_em;
    double* t_em;
    double* g_em;
    double* intensity;
    double* intensity_n;
    int32_t* attempts;
};

// Zeroes queue[0..n).  A small fill kernel, not a memset, so that the call can
// be captured into a graph and replayed.
hipError_t launch_zero(unsigned long long* queue, int32_t n, hipStream_t stream);

// Work distribution of the persistent trace kernels: pixels are handed out in
// chunks of `chunk` consecutive ordinals, ordinals enumerate the screen in
// tiles of tile_w x tile_h pixels (tile_w = nx, tile_h = 1 is row-major).
struct LaunchShape {
    int32_t chunk;
    int32_t tile_w;
    int32_t tile_h;
};

// Launches the persistent single-image trace kernel of c.metric on `grid`
// blocks of kBlock threads; *queue must be zero when the kernel starts.
hipError_t launch_trace(const ImageConst& c, const OutPtrs& o, unsigned long long* queue,
                        const LaunchShape& shape, int32_t grid, hipStream_t stream);

// Launches the persistent batched trace kernel over n_images images.  table,
// outs and chunk_start (n_images + 1 prefix sums of chunks per image) are
// device arrays in the kernel's image order; *queue must be zero.
hipError_t launch_trace_batch(const ImageConst* table, const OutPtrs* outs,
                              const int64_t* chunk_start, int32_t n_images,
                              unsigned long long* queue, const LaunchShape& shape, int32_t grid,
                              hipStream_t stream);

// LDS bytes of the batched kernel for n_images images.
size_t batch_lds_bytes(int32_t n_images);

// Resident blocks per compute unit of the single-image kernel of a metric and
// of the batched kernel.
int max_blocks_per_cu(int metric);
int max_batch_blocks_per_cu(int32_t n_images);

// Flux and intensity-weighted centroid of an image (Sec. 6.2): out[0..2] =
// {F, X_c, Y_c}.  `partials` is device scratch of 3 * kReduceBlocks doubles.
// Deterministic summation order.
constexpr int kReduceBlocks = 256;
hipError_t launch_reduce(const ImageConst& c, const double* intensity, double* partials,
                         double* out, hipStream_t stream);

}  // namespace rt
