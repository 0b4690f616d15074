// rt_kernels.h -- host-visible launch interface of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rt_device.h"

struct rt_scan_point;   // include/rt.h

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

// Work distribution of the persistent trace kernels.  With `order` null,
// pixels are handed out in chunks of `chunk` consecutive ordinals, ordinals
// enumerating the screen in tiles of tile_w x tile_h pixels (tile_w = nx,
// tile_h = 1 is row-major).  With `order` set (n_tiles tile indices, row-major
// tile numbering), a claim takes one whole tile, tiles in that order.
struct LaunchShape {
    int32_t chunk;
    int32_t tile_w;
    int32_t tile_h;
    const int32_t* order = nullptr;
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

// Launches the emission pass of an image after its trace (any kernel that
// traced it, in stream order): g_em, intensity_n and intensity from the
// ncross and r_em outputs, which must both be set.
hipError_t launch_emission(const ImageConst& c, const OutPtrs& o, hipStream_t stream);

// The emission pass of n_images images of a batch (device tables as for
// launch_trace_batch; max_pix the largest image).
hipError_t launch_emission_batch(const ImageConst* table, const OutPtrs* outs, int32_t n_images,
                                 int64_t max_pix, hipStream_t stream);

// Thick-disc trace of one image (rt_trace_thick): as launch_trace, with
// o.intensity the thick disc's intensity; *queue must be zero.
int thick_blocks_per_cu(int metric);
hipError_t launch_trace_thick(const ImageConst& c, const OutPtrs& o, unsigned long long* queue,
                              const LaunchShape& shape, int32_t grid, hipStream_t stream);

// Parameter scan (rt_parameter_scan): out[4i..4i+4) for pts[i].
hipError_t launch_scan(const ::rt_scan_point* pts, int32_t n, double* out, hipStream_t stream);

// Image diagnostics of `intensity` on the screen of c (rt_image_diagnostics):
// out[0..14); profile[n_bins] (or work memory when null); `work` holds
// diagnostics_scratch_doubles(n_bins) doubles, every one written before it is
// read (nothing needs clearing).  Deterministic.
size_t diagnostics_scratch_doubles(int32_t n_bins);
hipError_t launch_diagnostics(const ImageConst& c, const double* intensity, double bw,
                              int32_t n_bins, double* out, double* profile, double* work,
                              hipStream_t stream);
// The diagnostics' file-scope device work array for the entry point that
// allocates nothing: its device address on the current device (looked up
// once per device) and its size in doubles.
constexpr int32_t kNoAllocMaxBins = 65536;
hipError_t diagnostics_static_work(double** ptr, size_t* doubles);
// delta[i] = (q[i] - ref[i]) / ref[i] for i < n (rt_relative_deviation).
hipError_t launch_relative(const double* q, const double* ref, int32_t n, double* delta,
                           hipStream_t stream);

// Shadow-boundary search: `samples` (64, 32 or 16) lanes per direction
// dirs[2i], dirs[2i+1] (cos psi, sin psi); out[2i], out[2i+1] = the final bracket of b, status[i]
// = 0, or 1 (bracket left as given) when the ray at b_lo escapes or the one at
// b_hi does not; attempts[i] (if non-null) = the direction's step attempts.
hipError_t launch_boundary(const ImageConst& c, const double* dirs, int32_t n, int32_t samples,
                           double b_lo, double b_hi, double b_tol, double* out, int32_t* status,
                           int64_t* attempts, hipStream_t stream);

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

// Normalised visibility amplitudes (Sec. 6.4) of n_img images in one launch
// sequence.  VisImage holds one image (device pointers I [ny][nx], uv [K][2],
// amp [K] or null, vis [K][2] or null; the screen of its pixel centres);
// vis_layout fills the work-item and partial-sum offsets of a host table and
// returns the totals.  launch_visibility runs the flux partials (fpart:
// kVisFluxBlocks doubles per image), the partial sums (part: n_part double2)
// and the finish on the device copy d_tab of that table; max_k is the
// largest K.  Deterministic.
constexpr int kVisCols = 16;          // image columns per work item
constexpr int kVisFluxBlocks = 64;    // flux partials per image
struct VisImage {
    const double* I;
    const double* uv;
    double* amp;
    double* vis;
    int32_t nx, ny, K;
    int32_t nkg, ncb;                 // point groups of 64, column blocks of kVisCols
    int32_t item0;                    // first work item (wavefront) of the image
    int64_t part0;                    // first partial sum: [ncb][K]
    double x0, dx, y0, dy;
};
void vis_layout(VisImage* tab, int32_t n_img, int32_t* n_items, int64_t* n_part);
hipError_t launch_visibility(const VisImage* d_tab, int32_t n_img, int32_t n_items, int32_t max_k,
                             double2* part, double* fpart, hipStream_t stream);
// Points on n_q rings (radius q[j], device) at n_angles angles 2 pi a / n_angles:
// uv [n_q n_angles][2]; and the average of amp over each ring's angles (avg)
// with its amplitude at angle 0 (cut), either output optional.
hipError_t launch_ring_points(const double* q, int32_t n_q, int32_t n_angles, double* uv,
                              hipStream_t stream);
hipError_t launch_ring_average(const double* amp, int32_t n_q, int32_t n_angles, double* avg,
                               double* cut, hipStream_t stream);

// Mixed precision.  trace32: the binary32 pass over the screen (order of
// `shape`); rays leaving binary32 append a record of mixed_record_bytes() to
// `records` (room for n_pix) and bump counters[0] (records) and counters[1]
// (of which traced again from the screen); counters (32 u32: [0], [1], then
// u64 totals of step attempts at u32 offsets 4 (binary32) and 6 (binary64))
// and *queue start at 0.  resume: the binary64 pass over the counters[0]
// records (count read on the device); a continued ray reaching two crossings
// is traced again from the screen and counted in counters[1].
// copy_counters: stats[0..4) = {counters[0], counters[1], binary32 attempts,
// binary64 attempts}.  `pass` of mixed_blocks_per_cu: 0 trace32, 1 resume.
size_t mixed_record_bytes();
hipError_t launch_trace32(const ImageConst& c, const OutPtrs& o, unsigned long long* queue,
                          const LaunchShape& shape, int32_t grid, double* records,
                          unsigned int* counters, hipStream_t stream);
hipError_t launch_resume(const ImageConst& c, const OutPtrs& o, const double* records,
                         unsigned int* counters, unsigned long long* queue, int32_t chunk,
                         int32_t grid, hipStream_t stream);
hipError_t launch_copy_counters(const unsigned int* counters, long long* stats,
                                hipStream_t stream);
int mixed_blocks_per_cu(int metric, int pass);

// Image gradient (reverse mode through every ray's discrete map), with
// checkpointed recomputation:
//   forward:  for each pixel with dl_dI != 0 (screen order of `shape`), traces
//             the ray and stores a checkpoint (kVjpCkptDoubles) of its state
//             before every kseg-th accepted step into its `slots` slots at
//             ckpt + pix * slots checkpoints (kseg starts at kVjpSeg and
//             doubles, the slots thinned to every other one, whenever they
//             run out); count[pix] = accepted steps up to the last emitting
//             crossing (0 if none), kseg[pix] = the final interval;
//             counters[0] += rays with count > 0, counters[1] += their counts;
//   backward: for those pixels, restores each segment's checkpoint from the
//             last to the first, recomputes its steps (at most kVjpBuf at a
//             time, into the calling lane's buffer of kVjpBuf records of
//             kVjpRecBytes at lane_buf + global thread index * kVjpBuf
//             records) and reverses them, then writes grad_pix[pix][4] = dL/dq
//             with jac[m][j] the derivative of per-ray parameter m along the
//             image parameter q_j.
// Each pass needs its zeroed queue counter; `grid` blocks of kBlock threads
// (the backward pass's lane buffers must cover grid * kBlock lanes).
// The backward pass adds 1 to counters[2] for a recomputation that ended
// before its steps (never, unless it diverged from the trace; it then stops).
// `pass` of vjp_blocks_per_cu: 0 forward, 1 backward.  copy_vjp_stats:
// stats[0..3) = counters[0..3).
constexpr int kVjpPrims = 11;
constexpr int kVjpRecBytes = 240;
constexpr int kVjpCkptDoubles = 16;
constexpr int kVjpSeg = 32;     // accepted steps per segment before any thinning
constexpr int kVjpBuf = 32;     // step records recomputed at a time
constexpr int kGradBlocks = 256;
hipError_t launch_vjp_forward(const ImageConst& c, const double* dl_dI, int32_t slots,
                              double* ckpt, int32_t* count, int32_t* kseg,
                              unsigned long long* counters, unsigned long long* queue,
                              const LaunchShape& shape, int32_t grid, hipStream_t stream);
hipError_t launch_vjp_backward(const ImageConst& c, const double* dl_dI, const int32_t* count,
                               const int32_t* kseg, int32_t slots, const double* ckpt,
                               double* lane_buf, const double (&jac)[kVjpPrims][4],
                               double* grad_pix, unsigned long long* counters,
                               unsigned long long* queue, const LaunchShape& shape, int32_t grid,
                               hipStream_t stream);
hipError_t launch_copy_vjp_stats(const unsigned long long* counters, long long* stats,
                                 hipStream_t stream);
int vjp_blocks_per_cu(int metric, int pass);
// p[0..n) = 0 (a fill kernel).
hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t stream);
// grad[0..4) = sum over pixels of grad_pix[pix][0..4), in a fixed order;
// `partials` holds 4 kGradBlocks doubles.
hipError_t launch_grad_reduce(const double* grad_pix, int64_t n_pix, double* partials,
                              double* grad, hipStream_t stream);

}  // namespace rt
