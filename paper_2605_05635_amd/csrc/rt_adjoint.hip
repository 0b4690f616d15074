// rt_adjoint.hip -- gfx950 kernels of the image gradient: reverse mode
// through the computed discrete map of every ray (the per-ray pieces are in
// rt_vjp.h), with checkpointed recomputation so that memory grows with the
// number of checkpoints, not of steps.  Two persistent passes, each lane
// owning one ray at a time:
//
//  1. forward:  trace every pixel whose loss cotangent is non-zero and store a
//               checkpoint of the ray before every kVjpSeg-th accepted step
//               (a fixed number of slots per pixel: when they run out the
//               interval doubles and every other checkpoint is dropped); record
//               how many steps matter -- up to and including the last one whose
//               crossing emits (nothing after it reaches the intensity);
//  2. backward: for each segment from the last to the first, restore its
//               checkpoint, recompute its accepted steps (with their stage
//               derivatives) into the lane's buffer -- at most kVjpBuf at a time,
//               taken from the segment's end -- and reverse them with
//               reverse_step; finally chain the adjoint of the initial state
//               through the screen map into the pixel's four gradient terms.
//
// The recomputation repeats the forward pass's attempts exactly (the same
// code on the same state), so the steps reversed are the steps traced.  Within
// a wavefront the lanes recompute together, then reverse together (two
// ballot-driven phases per round), so the two kinds of work do not interleave
// instruction by instruction.  A last pair of kernels sums the per-pixel
// gradients in a fixed order.  No pass needs a result on the host.
#include "rt_vjp.h"

namespace rt {
namespace {

using namespace ray;
using vjp::kRecDoubles;

static_assert(vjp::kPrims == kVjpPrims, "parameter-adjoint count");
static_assert(kRecDoubles * 8 == kVjpRecBytes, "tape record size");
static_assert(vjp::kCkptDoubles == kVjpCkptDoubles, "checkpoint size");
static_assert(kVjpSeg % kVjpBuf == 0, "segments split into whole buffers");

// Adds the wave's sums of a and b to total[0], total[1] (lane 0; converged).
__device__ __forceinline__ void add_wave_totals(uint32_t a, uint32_t b,
                                                unsigned long long* total) {
    unsigned long long x = a, y = b;
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off);
        y += __shfl_xor(y, off);
    }
    if (__lane_id() == 0 && (x | y) != 0ull) {
        atomicAdd(&total[0], x);
        atomicAdd(&total[1], y);
    }
}

// Pass 1.
template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void vjp_forward_kernel(
    ImageConst c, const double* __restrict__ dl_dI, int32_t slots, double* __restrict__ ckpt,
    int32_t* __restrict__ count, int32_t* __restrict__ kseg, unsigned long long* counters,
    unsigned long long* queue, LaunchShape shape) {
    const Hot k = hot_of(c);
    const OutPtrs none{};
    Ray r;
    int32_t acc = 0, last = -1, K = kVjpSeg, used = 0;
    double* mine = ckpt;
    bool live = false;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    TileClaim tc{0, 0, 1, 1.0f};
    uint32_t rays = 0, steps = 0;
    auto claim = [&]() { return claim_screen(shape, c.nx, c.ny, queue, next, end, tc); };
    auto take = [&](int64_t ordinal) {
        const int64_t pix = claimed_pixel(shape, c.nx, c.ny, tc, ordinal);
        start_ray<METRIC>(c, k, pix, r);
        acc = 0;
        last = -1;
        K = kVjpSeg;
        live = dl_dI[pix] != 0.0;
        mine = ckpt + pix * static_cast<int64_t>(slots) * kVjpCkptDoubles;
        if (live) vjp::store_checkpoint(mine, r, 0);
        used = 1;
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            bool done = !live;
            if (live) {
                const int32_t n0 = r.ncross;
                const int32_t st = attempt<METRIC>(k, none, c.n_pix, r);
                if (st != RAY_STEP_LIMIT && r.after_reject == 0) {   // accepted
                    if (r.ncross != n0 && n0 < 3) {
                        const double Rc = n0 == 0 ? r.rc[0] : (n0 == 1 ? r.rc[1] : r.rc[2]);
                        if (vjp::emits<METRIC>(c, k, Rc, r.E, r.L)) last = acc;
                    }
                    ++acc;
                    if (st == 0 && r.ncross < 3 && acc % K == 0) {
                        if (used == slots) {   // out of slots: keep every other one
                            for (int32_t i = 1; i < slots / 2; ++i)
                                for (int j = 0; j < kVjpCkptDoubles; ++j)
                                    mine[i * kVjpCkptDoubles + j] = mine[2 * i * kVjpCkptDoubles + j];
                            used = slots / 2;
                            K *= 2;
                        }
                        vjp::store_checkpoint(mine + used * kVjpCkptDoubles, r, acc);
                        ++used;
                    }
                }
                done = st != 0 || r.ncross >= 3;
            }
            if (done) {
                count[r.pix] = last + 1;
                kseg[r.pix] = K;
                if (last >= 0) {
                    ++rays;
                    steps += static_cast<uint32_t>(last + 1);
                }
                active = false;
            }
        }
    }
    add_wave_totals(rays, steps, counters);
}

struct JacArg {
    double m[kVjpPrims][4];
};

// Pass 2.
template <int METRIC>
__global__ __launch_bounds__(kBlock) void vjp_backward_kernel(
    ImageConst c, const double* __restrict__ dl_dI, const int32_t* __restrict__ count,
    const int32_t* __restrict__ kseg, int32_t slots, const double* __restrict__ ckpt,
    double* __restrict__ lane_buf, JacArg J, double* __restrict__ grad_pix,
    unsigned long long* counters, unsigned long long* queue, LaunchShape shape) {
    const Hot k = hot_of(c);
    const OutPtrs none{};
    double* const buf = lane_buf + (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) *
                                       (static_cast<int64_t>(kVjpBuf) * kRecDoubles);
    Ray r;
    int64_t pix = 0;
    const double* mine = ckpt;
    int32_t K = kVjpSeg, seg = 0, seg_len = 0, chunk = 0, acc = 0, rec_lo = 0, rec_hi = 0;
    int32_t n_rec = 0;
    bool fwd = false;
    double E = 0.0, L = 0.0, Ib = 0.0;
    ScreenDir dir{0.0, 0.0, 0.0};
    double xb[4], Eb, Lb, pb[4], rinb;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    TileClaim tc{0, 0, 1, 1.0f};
    // (re)start the recomputation of chunk `chunk` of segment `seg`
    auto begin_chunk = [&]() {
        vjp::load_checkpoint<METRIC>(mine + seg * kVjpCkptDoubles, k, E, L, pix, r);
        acc = 0;
        rec_lo = chunk * kVjpBuf;
        rec_hi = rec_lo + kVjpBuf < seg_len ? rec_lo + kVjpBuf : seg_len;
        n_rec = 0;
        fwd = true;
    };
    auto claim = [&]() { return claim_screen(shape, c.nx, c.ny, queue, next, end, tc); };
    auto take = [&](int64_t ordinal) {
        pix = claimed_pixel(shape, c.nx, c.ny, tc, ordinal);
        const int32_t cnt = count[pix];
        fwd = false;
        n_rec = 0;
        if (cnt <= 0) return;   // nothing reaches the intensity: the zero gradient stands
        dir = screen_dir(c, pix);
        E = c.obs_N - c.obs_gTph_over_sq_gphph * dir.nph;
        L = c.obs_sq_gphph * dir.nph;
        Ib = dl_dI[pix];
        for (int i = 0; i < 4; ++i) {
            xb[i] = 0.0;
            pb[i] = 0.0;
        }
        Eb = Lb = rinb = 0.0;
        K = kseg[pix];
        mine = ckpt + pix * static_cast<int64_t>(slots) * kVjpCkptDoubles;
        seg = (cnt - 1) / K;
        seg_len = cnt - seg * K;
        chunk = (seg_len - 1) / kVjpBuf;
        begin_chunk();
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active && !fwd && n_rec == 0) active = false;   // an empty ray
        // Recompute: the lanes with a chunk to fill run attempts, recording the
        // accepted steps rec_lo..rec_hi-1 of their segment.
        while (__ballot(active && fwd) != 0ull) {
            if (active && fwd) {
                double* slot = buf + n_rec * kRecDoubles;
                const double x0 = r.y[1], x1 = r.y[2], x2 = r.y[4], x3 = r.y[5], h = r.h;
                const int32_t n0 = r.ncross;
                const int32_t st = attempt<METRIC>(k, none, c.n_pix, r, vjp::TapeStages{slot});
                if (st != RAY_STEP_LIMIT && r.after_reject == 0) {   // accepted
                    if (acc >= rec_lo) {
                        const bool crossed = r.ncross != n0 && n0 < 3;
                        double2* p = reinterpret_cast<double2*>(slot);
                        p[0] = make_double2(x0, x1);
                        p[1] = make_double2(x2, x3);
                        p[2] = make_double2(h, crossed ? static_cast<double>(n0) : -1.0);
                        ++n_rec;
                    }
                    ++acc;
                    if (acc == rec_hi) fwd = false;
                }
                // The recomputation repeats the traced attempts, so the ray
                // cannot end before rec_hi; should it ever (a recomputation that
                // diverged from the trace), stop and count it rather than spin.
                if (fwd && st != 0) {
                    fwd = false;
                    atomicAdd(&counters[2], 1ull);
                }
            }
        }
        // Reverse: the lanes with recorded steps walk them backwards.
        while (__ballot(active && n_rec > 0) != 0ull) {
            if (active && n_rec > 0) {
                const double* rp = buf + (n_rec - 1) * kRecDoubles;
                const double2* p = reinterpret_cast<const double2*>(rp);
                const double2 a = p[0], b = p[1], hc = p[2];
                const double x0[4] = {a.x, a.y, b.x, b.y};
                double kin[24];
                const double2* q = reinterpret_cast<const double2*>(rp + vjp::kRecStages);
                for (int m = 0; m < 12; ++m) {
                    const double2 v = q[m];
                    kin[2 * m] = v.x;
                    kin[2 * m + 1] = v.y;
                }
                vjp::reverse_step<METRIC>(c, k, E, L, x0, hc.x, static_cast<int>(hc.y), kin, Ib,
                                          xb, Eb, Lb, pb, rinb);
                if (--n_rec == 0) {
                    if (chunk > 0) {
                        --chunk;
                        begin_chunk();
                    } else if (seg > 0) {
                        --seg;
                        seg_len = K;
                        chunk = K / kVjpBuf - 1;
                        begin_chunk();
                    } else {
                        // Initial state (0, R_o, theta_o, 0, sqrt(g_RR) n_R,
                        // sqrt(g_thth) n_theta), E = N_o - (g_Tphi/sqrt(g_phiphi)) n_phi,
                        // l = sqrt(g_phiphi) n_phi.
                        double prim[kVjpPrims];
                        prim[vjp::P_CHI] = pb[0];
                        prim[vjp::P_M0] = pb[1];
                        prim[vjp::P_M1] = pb[2];
                        prim[vjp::P_M2] = pb[3];
                        prim[vjp::P_RIN] = rinb;
                        prim[vjp::P_OBS_N] = Eb;
                        prim[vjp::P_OBS_TPH] = -Eb * dir.nph;
                        prim[vjp::P_OBS_PH] = Lb * dir.nph;
                        prim[vjp::P_OBS_R] = xb[2] * dir.nR;
                        prim[vjp::P_OBS_TH] = xb[3] * dir.nth;
                        prim[vjp::P_INCL] = xb[1];
                        for (int j = 0; j < 4; ++j) {
                            double g = 0.0;
                            for (int m = 0; m < kVjpPrims; ++m) g += prim[m] * J.m[m][j];
                            grad_pix[pix * 4 + j] = g;
                        }
                        active = false;
                    }
                }
            }
        }
    }
}

__global__ void copy_vjp_stats(const unsigned long long* __restrict__ counters,
                               long long* __restrict__ stats) {
    if (threadIdx.x < 3) stats[threadIdx.x] = static_cast<long long>(counters[threadIdx.x]);
}

__global__ void fill_zero(double* __restrict__ p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Gradient sum over pixels in a fixed order: block b adds the pixels
// [b n/B, (b+1) n/B) with a fixed tree in LDS; one block then adds the B
// partial sums in index order.
constexpr int kGradThreads = 256;

__global__ __launch_bounds__(kGradThreads) void grad_partial(const double* __restrict__ gp,
                                                             int64_t n_pix,
                                                             double* __restrict__ part) {
    __shared__ double sh[4][kGradThreads];
    const int64_t per = (n_pix + gridDim.x - 1) / gridDim.x;
    const int64_t lo = per * blockIdx.x;
    const int64_t hi = lo + per < n_pix ? lo + per : n_pix;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = lo + threadIdx.x; p < hi; p += kGradThreads)
        for (int j = 0; j < 4; ++j) acc[j] += gp[p * 4 + j];
    for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = kGradThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w)
            for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void grad_final(const double* __restrict__ part, int32_t nblocks,
                           double* __restrict__ grad) {
    const int j = threadIdx.x;
    if (j >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[b * 4 + j];
    grad[j] = s;
}

template <class Kern>
int occupancy(Kern kern, size_t lds = 0) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBlock, lds);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

hipError_t launch_vjp_forward(const ImageConst& c, const double* dl_dI, int32_t slots,
                              double* ckpt, int32_t* count, int32_t* kseg,
                              unsigned long long* counters, unsigned long long* queue,
                              const LaunchShape& shape, int32_t grid, hipStream_t stream) {
    if (c.metric == KERR)
        hipLaunchKernelGGL(vjp_forward_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, slots, ckpt, count, kseg, counters, queue, shape);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(vjp_forward_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, slots, ckpt, count, kseg, counters, queue, shape);
    else if (c.ex_near)
        hipLaunchKernelGGL(vjp_forward_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, slots, ckpt, count, kseg, counters, queue, shape);
    else
        hipLaunchKernelGGL(vjp_forward_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, slots, ckpt, count, kseg, counters, queue, shape);
    return hipGetLastError();
}

hipError_t launch_vjp_backward(const ImageConst& c, const double* dl_dI, const int32_t* count,
                               const int32_t* kseg, int32_t slots, const double* ckpt,
                               double* lane_buf, const double (&jac)[kVjpPrims][4],
                               double* grad_pix, unsigned long long* counters,
                               unsigned long long* queue, const LaunchShape& shape, int32_t grid,
                               hipStream_t stream) {
    JacArg J;
    for (int m = 0; m < kVjpPrims; ++m)
        for (int j = 0; j < 4; ++j) J.m[m][j] = jac[m][j];
    if (c.metric == KERR)
        hipLaunchKernelGGL(vjp_backward_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, count, kseg, slots, ckpt, lane_buf, J, grad_pix, counters, queue, shape);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(vjp_backward_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, count, kseg, slots, ckpt, lane_buf, J, grad_pix, counters, queue, shape);
    else if (c.ex_near)
        hipLaunchKernelGGL(vjp_backward_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream,
                           c, dl_dI, count, kseg, slots, ckpt, lane_buf, J, grad_pix, counters,
                           queue, shape);
    else
        hipLaunchKernelGGL(vjp_backward_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, count, kseg, slots, ckpt, lane_buf, J, grad_pix, counters, queue, shape);
    return hipGetLastError();
}

hipError_t launch_copy_vjp_stats(const unsigned long long* counters, long long* stats,
                                 hipStream_t stream) {
    hipLaunchKernelGGL(copy_vjp_stats, dim3(1), dim3(64), 0, stream, counters, stats);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                       stream, p, n);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double* grad_pix, int64_t n_pix, double* partials,
                              double* grad, hipStream_t stream) {
    hipLaunchKernelGGL(grad_partial, dim3(kGradBlocks), dim3(kGradThreads), 0, stream, grad_pix,
                       n_pix, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(grad_final, dim3(1), dim3(64), 0, stream, partials, kGradBlocks, grad);
    return hipGetLastError();
}

int vjp_blocks_per_cu(int metric, int pass) {
    if (pass == 0) {
        if (metric == KERR) return occupancy(vjp_forward_kernel<KERR>);
        if (metric == EINASTO) return occupancy(vjp_forward_kernel<EINASTO>);
        return occupancy(vjp_forward_kernel<CNFW>);
    }
    if (metric == KERR) return occupancy(vjp_backward_kernel<KERR>);
    if (metric == EINASTO) return occupancy(vjp_backward_kernel<EINASTO>);
    return occupancy(vjp_backward_kernel<CNFW>);
}

}  // namespace rt
