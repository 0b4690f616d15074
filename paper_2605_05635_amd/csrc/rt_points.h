// rt_points.h -- host-visible launch interface of the kernels that trace
// listed screen points and refine the screen near the lensing-band
// boundaries (rt_points.hip).
#pragma once

#include "rt_kernels.h"

namespace rt {

// Resident workgroups per compute unit of the point trace for `metric`.
int points_blocks_per_cu(int metric);

// Traces the c.n_pix points xy[2 i], xy[2 i + 1] (X_i, Y_i) of the screen of
// c, ray i recorded as "pixel" i of o (crossing records [3][n_pix], NaN past
// min(N_cross, 3)), then, when c.emission, the emission of its records.
// *queue must be zero; `grid` blocks of kBlock threads.
hipError_t launch_trace_points(const ImageConst& c, const double* xy, const OutPtrs& o,
                               unsigned long long* queue, int32_t grid, hipStream_t stream);

// Screen refinement of an nx x ny screen whose N_cross and status maps are
// ncross and status: marks the pixels with a 4-neighbour of another N_cross or
// status; writes the count to *n_marked, and for the first max_marked marked
// pixels in pixel order (m = 0, 1, ...) pix[m] (when pix is set) and the
// sub x sub subpixel centres xy[2 (m sub^2 + b sub + a) + {0, 1}] =
// (x0 + (ix + (a + 1/2)/sub) dx, y0 + (iy + (b + 1/2)/sub) dy).
// block_count: scratch of (n_pix + kBlock - 1)/kBlock int64.
hipError_t launch_refine(const ImageConst& c, const uint8_t* ncross, const uint8_t* status,
                         int32_t sub, int64_t max_marked, double* xy, int64_t* pix,
                         int64_t* n_marked, int64_t* block_count, hipStream_t stream);

}  // namespace rt
