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

// Launches the persistent trace kernel of c.metric on `grid` blocks of kBlock
// threads, wavefronts claiming `chunk` pixels at a time from *queue (which must
// be zero when the kernel starts).
hipError_t launch_trace(const ImageConst& c, const OutPtrs& o, unsigned long long* queue,
                        int32_t chunk, int32_t grid, hipStream_t stream);

// Resident blocks of the trace kernel per compute unit.
int max_blocks_per_cu(int metric);

// Flux and intensity-weighted centroid of an image (Sec. 6.2): out[0..2] =
// {F, X_c, Y_c}.  `partials` is device scratch of 3 * kReduceBlocks doubles.
// Deterministic summation order.
constexpr int kReduceBlocks = 256;
hipError_t launch_reduce(const ImageConst& c, const double* intensity, double* partials,
                         double* out, hipStream_t stream);

}  // namespace rt
