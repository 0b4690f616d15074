// rt_adjoint.hip -- gfx950 kernels of the image gradient: reverse mode
// through the computed discrete map of every ray (the per-ray pieces are in
// rt_vjp.h).  Two persistent passes, each lane owning one ray at a time:
//
//  1. tape:    trace every pixel whose loss cotangent is non-zero, writing each
//              accepted step's start state, size and crossing index into the
//              pixel's own tape region (cap steps), and record how many steps
//              matter: up to and including the last one whose crossing emits
//              (nothing after it reaches the intensity).  A ray that needs
//              more than cap steps is marked (count -1) and counted;
//  2. reverse: walk each tape backwards with reverse_step, then chain the
//              adjoint of the initial state through the screen map and write
//              the pixel's gradient along the four image parameters.
//
// The marked rays (rare: long photon-ring orbits) go through a list-driven
// variant of the same passes, with tapes sized exactly by a counting pass and
// packed longest first.  The tape holds each step's stage derivatives as well
// (240 bytes per step), so that the reverse pass does not recompute the six
// right-hand sides of a step (measured 5 % faster per gradient than a 48-byte
// tape with recomputation).  A last pair of kernels sums the per-pixel
// gradients in a fixed order.
#include "rt_vjp.h"

namespace rt {
namespace {

using namespace ray;
using vjp::kRecDoubles;

static_assert(vjp::kPrims == kVjpPrims, "parameter-adjoint count");
static_assert(kRecDoubles * 8 == kVjpRecBytes, "tape record size");

struct ListShape {
    int32_t chunk;
};

template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void vjp_count_kernel(
    ImageConst c, const double* __restrict__ dl_dI, int32_t* __restrict__ count,
    unsigned long long* queue, LaunchShape shape) {
    // Only the pixels whose count is -1 on entry are traced (the rays the
    // dense tape could not hold); every other count is set to 0.
    const Hot k = hot_of(c);
    const OutPtrs none{};
    Ray r;
    int32_t acc = 0, last = -1;
    bool live = false;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    TileClaim tc{0, 0, 1};
    auto claim = [&]() { return claim_screen(shape, c.nx, c.ny, queue, next, end, tc); };
    auto take = [&](int64_t ordinal) {
        const int64_t pix = claimed_pixel(shape, c.nx, c.ny, tc, ordinal);
        start_ray<METRIC>(c, k, pix, r);
        acc = 0;
        last = -1;
        live = count[pix] < 0 && dl_dI[pix] != 0.0;
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            bool done = !live;
            if (live) {
                const int32_t n0 = r.ncross;
                const int32_t st = attempt<METRIC>(k, none, c.n_pix, r);
                if (st != RAY_STEP_LIMIT && r.after_reject == 0) {
                    if (r.ncross != n0 && n0 < 3) {
                        const double Rc = n0 == 0 ? r.rc[0] : (n0 == 1 ? r.rc[1] : r.rc[2]);
                        if (vjp::emits<METRIC>(c, k, Rc, r.E, r.L)) last = acc;
                    }
                    ++acc;
                }
                done = st != 0 || r.ncross >= 3;
            }
            if (done) {
                count[r.pix] = last + 1;
                active = false;
            }
        }
    }
}

template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void vjp_tape_kernel(
    ImageConst c, const int32_t* __restrict__ list_pix, const int64_t* __restrict__ list_off,
    const int32_t* __restrict__ count, int64_t n_list, int64_t rec_base,
    double* __restrict__ tape, int32_t* __restrict__ taped, unsigned long long* queue,
    ListShape shape) {
    const Hot k = hot_of(c);
    const OutPtrs none{};
    Ray r;
    int64_t entry = 0, rec = 0;
    int32_t acc = 0, want = 0;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    auto claim = [&]() { return claim_chunk(queue, shape.chunk, n_list, next, end); };
    auto take = [&](int64_t e) {
        entry = e;
        const int64_t pix = list_pix[e];
        start_ray<METRIC>(c, k, pix, r);
        rec = list_off[e] - rec_base;
        want = count[pix];
        acc = 0;
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            const double x0 = r.y[1], x1 = r.y[2], x2 = r.y[4], x3 = r.y[5], h = r.h;
            const int32_t n0 = r.ncross;
            double* const slot = tape + (rec + acc) * kRecDoubles;
            const int32_t st = attempt<METRIC>(k, none, c.n_pix, r, vjp::TapeStages{slot});
            if (st != RAY_STEP_LIMIT && r.after_reject == 0) {
                double2* p = reinterpret_cast<double2*>(slot);
                const double cross = (r.ncross != n0 && n0 < 3) ? static_cast<double>(n0) : -1.0;
                p[0] = make_double2(x0, x1);
                p[1] = make_double2(x2, x3);
                p[2] = make_double2(h, cross);
                ++acc;
            }
            if (acc >= want || st != 0) {
                taped[entry] = acc;
                active = false;
            }
        }
    }
}

// Pass 1 of the common path.  counters[0] += marked rays, counters[1] += rays
// with a non-zero count, counters[2] += their steps (one atomic per wave each).
template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void vjp_tape_dense_kernel(
    ImageConst c, const double* __restrict__ dl_dI, int32_t cap, double* __restrict__ tape,
    double* overflow, int32_t* __restrict__ count, unsigned int* counters,
    unsigned long long* queue, LaunchShape shape) {
    const Hot k = hot_of(c);
    const OutPtrs none{};
    Ray r;
    int32_t acc = 0, last = -1;
    bool live = false;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    TileClaim tc{0, 0, 1};
    auto claim = [&]() { return claim_screen(shape, c.nx, c.ny, queue, next, end, tc); };
    auto take = [&](int64_t ordinal) {
        const int64_t pix = claimed_pixel(shape, c.nx, c.ny, tc, ordinal);
        start_ray<METRIC>(c, k, pix, r);
        acc = 0;
        last = -1;
        live = dl_dI[pix] != 0.0;
    };
    const int lane = __lane_id();
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        int32_t finished = 0;   // 0: none; 1: counted ray; 2: marked ray
        int32_t nsteps = 0;
        if (active) {
            bool done = !live;
            if (live) {
                const double x0 = r.y[1], x1 = r.y[2], x2 = r.y[4], x3 = r.y[5], h = r.h;
                const int32_t n0 = r.ncross;
                // steps past the pixel's region write their stages to a scratch
                // record that nothing reads (a branch-free store target)
                double* const slot =
                    acc < cap ? tape + (r.pix * static_cast<int64_t>(cap) + acc) * kRecDoubles
                              : overflow;
                const int32_t st = attempt<METRIC>(k, none, c.n_pix, r, vjp::TapeStages{slot});
                if (st != RAY_STEP_LIMIT && r.after_reject == 0) {
                    const bool crossed = r.ncross != n0 && n0 < 3;
                    if (acc < cap) {
                        double2* p = reinterpret_cast<double2*>(slot);
                        p[0] = make_double2(x0, x1);
                        p[1] = make_double2(x2, x3);
                        p[2] = make_double2(h, crossed ? static_cast<double>(n0) : -1.0);
                    }
                    if (crossed) {
                        const double Rc = n0 == 0 ? r.rc[0] : (n0 == 1 ? r.rc[1] : r.rc[2]);
                        if (vjp::emits<METRIC>(c, k, Rc, r.E, r.L)) last = acc;
                    }
                    ++acc;
                }
                done = st != 0 || r.ncross >= 3;
            }
            if (done) {
                nsteps = last + 1;
                if (nsteps > cap) {
                    count[r.pix] = -1;
                    finished = 2;
                } else {
                    count[r.pix] = nsteps;
                    finished = nsteps > 0 ? 1 : 0;
                }
                active = false;
            }
        }
        const unsigned long long mark = __ballot(finished == 2);
        const unsigned long long kept = __ballot(finished == 1);
        if ((mark | kept) != 0ull) {
            unsigned int s = finished == 1 ? static_cast<unsigned int>(nsteps) : 0u;
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (lane == 0) {
                if (mark) atomicAdd(&counters[0], static_cast<unsigned int>(__popcll(mark)));
                if (kept) {
                    atomicAdd(&counters[1], static_cast<unsigned int>(__popcll(kept)));
                    atomicAdd(&counters[2], s);
                }
            }
        }
    }
}

struct JacArg {
    double m[kVjpPrims][4];
};

// Pass 2.  DENSE: items are the screen's pixels in the order of `shape`, the
// pixel's tape at pix * cap records, steps[pix] of them (none if <= 0).
// Otherwise items are list entries: pixel list_pix[e], tape at list_off[e] -
// rec_base, steps[e] records.
template <int METRIC, bool DENSE>
__global__ __launch_bounds__(kBlock) void vjp_reverse_kernel(
    ImageConst c, const double* __restrict__ dl_dI, const int32_t* __restrict__ list_pix,
    const int64_t* __restrict__ list_off, const int32_t* __restrict__ steps, int64_t n_items,
    int64_t rec_base, int32_t cap, const double* __restrict__ tape, JacArg J,
    double* __restrict__ grad_pix, unsigned long long* queue, LaunchShape shape) {
    const Hot k = hot_of(c);
    int64_t pix = 0, rec = 0;
    int32_t step = 0;
    bool skip = false;
    double E = 0.0, L = 0.0, Ib = 0.0;
    ScreenDir dir{0.0, 0.0, 0.0};
    double xb[4], Eb, Lb, pb[4], rinb;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    TileClaim tc{0, 0, 1};
    auto claim = [&]() {
        if constexpr (DENSE) return claim_screen(shape, c.nx, c.ny, queue, next, end, tc);
        return claim_chunk(queue, shape.chunk, n_items, next, end);
    };
    auto take = [&](int64_t e) {
        if constexpr (DENSE) {
            pix = claimed_pixel(shape, c.nx, c.ny, tc, e);
            rec = pix * static_cast<int64_t>(cap);
            step = steps[pix] - 1;
        } else {
            pix = list_pix[e];
            rec = list_off[e] - rec_base;
            step = steps[e] - 1;
        }
        skip = step < 0;
        dir = screen_dir(c, pix);
        E = c.obs_N - c.obs_gTph_over_sq_gphph * dir.nph;
        L = c.obs_sq_gphph * dir.nph;
        Ib = dl_dI[pix];
        for (int i = 0; i < 4; ++i) {
            xb[i] = 0.0;
            pb[i] = 0.0;
        }
        Eb = Lb = rinb = 0.0;
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            if (step >= 0) {
                const double* rp = tape + (rec + step) * kRecDoubles;
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
                --step;
            }
            if (step < 0 && skip) {
                active = false;   // no step matters: the zero-filled gradient stands
            } else if (step < 0) {
                // Initial state (0, R_o, theta_o, 0, sqrt(g_RR) n_R, sqrt(g_thth) n_theta),
                // E = N_o - (g_Tphi/sqrt(g_phiphi)) n_phi, l = sqrt(g_phiphi) n_phi.
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

hipError_t launch_vjp_count(const ImageConst& c, const double* dl_dI, int32_t* count,
                            unsigned long long* queue, const LaunchShape& shape, int32_t grid,
                            hipStream_t stream) {
    if (c.metric == KERR)
        hipLaunchKernelGGL(vjp_count_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c, dl_dI,
                           count, queue, shape);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(vjp_count_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, count, queue, shape);
    else if (c.ex_near)
        hipLaunchKernelGGL(vjp_count_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream, c, dl_dI,
                           count, queue, shape);
    else
        hipLaunchKernelGGL(vjp_count_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c, dl_dI,
                           count, queue, shape);
    return hipGetLastError();
}

hipError_t launch_vjp_tape(const ImageConst& c, const int32_t* list_pix, const int64_t* list_off,
                           const int32_t* count, int64_t n_list, int64_t rec_base, double* tape,
                           int32_t* taped, unsigned long long* queue, int32_t chunk,
                           int32_t grid, hipStream_t stream) {
    const ListShape sh{chunk};
    if (c.metric == KERR)
        hipLaunchKernelGGL(vjp_tape_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           list_pix, list_off, count, n_list, rec_base, tape, taped, queue, sh);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(vjp_tape_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c,
                           list_pix, list_off, count, n_list, rec_base, tape, taped, queue, sh);
    else if (c.ex_near)
        hipLaunchKernelGGL(vjp_tape_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           list_pix, list_off, count, n_list, rec_base, tape, taped, queue, sh);
    else
        hipLaunchKernelGGL(vjp_tape_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c,
                           list_pix, list_off, count, n_list, rec_base, tape, taped, queue, sh);
    return hipGetLastError();
}

hipError_t launch_vjp_tape_dense(const ImageConst& c, const double* dl_dI, int32_t cap,
                                 double* tape, double* overflow, int32_t* count,
                                 unsigned int* counters,
                                 unsigned long long* queue, const LaunchShape& shape,
                                 int32_t grid, hipStream_t stream) {
    if (c.metric == KERR)
        hipLaunchKernelGGL(vjp_tape_dense_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, cap, tape, overflow, count, counters, queue, shape);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(vjp_tape_dense_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, cap, tape, overflow, count, counters, queue, shape);
    else if (c.ex_near)
        hipLaunchKernelGGL(vjp_tape_dense_kernel<CNFW_NEAR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, cap, tape, overflow, count, counters, queue, shape);
    else
        hipLaunchKernelGGL(vjp_tape_dense_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, cap, tape, overflow, count, counters, queue, shape);
    return hipGetLastError();
}

namespace {
template <bool DENSE>
hipError_t reverse_launch(const ImageConst& c, const double* dl_dI, const int32_t* list_pix,
                          const int64_t* list_off, const int32_t* steps, int64_t n_items,
                          int64_t rec_base, int32_t cap, const double* tape,
                          const double (&jac)[kVjpPrims][4], double* grad_pix,
                          unsigned long long* queue, const LaunchShape& shape, int32_t grid,
                          hipStream_t stream) {
    JacArg J;
    for (int m = 0; m < kVjpPrims; ++m)
        for (int j = 0; j < 4; ++j) J.m[m][j] = jac[m][j];
    if (c.metric == KERR)
        hipLaunchKernelGGL((vjp_reverse_kernel<KERR, DENSE>), dim3(grid), dim3(kBlock),
                           0, stream, c, dl_dI, list_pix, list_off, steps, n_items,
                           rec_base, cap, tape, J, grad_pix, queue, shape);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL((vjp_reverse_kernel<EINASTO, DENSE>), dim3(grid), dim3(kBlock),
                           0, stream, c, dl_dI, list_pix, list_off, steps, n_items,
                           rec_base, cap, tape, J, grad_pix, queue, shape);
    else if (c.ex_near)
        hipLaunchKernelGGL((vjp_reverse_kernel<CNFW_NEAR, DENSE>), dim3(grid), dim3(kBlock),
                           0, stream, c, dl_dI, list_pix, list_off, steps, n_items,
                           rec_base, cap, tape, J, grad_pix, queue, shape);
    else
        hipLaunchKernelGGL((vjp_reverse_kernel<CNFW, DENSE>), dim3(grid), dim3(kBlock),
                           0, stream, c, dl_dI, list_pix, list_off, steps, n_items,
                           rec_base, cap, tape, J, grad_pix, queue, shape);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_vjp_reverse(const ImageConst& c, const double* dl_dI, const int32_t* list_pix,
                              const int64_t* list_off, const int32_t* taped, int64_t n_list,
                              int64_t rec_base, const double* tape,
                              const double (&jac)[kVjpPrims][4], double* grad_pix,
                              unsigned long long* queue, int32_t chunk, int32_t grid,
                              hipStream_t stream) {
    return reverse_launch<false>(c, dl_dI, list_pix, list_off, taped, n_list, rec_base, 0, tape,
                                 jac, grad_pix, queue, LaunchShape{chunk, 1, 1}, grid, stream);
}

hipError_t launch_vjp_reverse_dense(const ImageConst& c, const double* dl_dI,
                                    const int32_t* count, int32_t cap, const double* tape,
                                    const double (&jac)[kVjpPrims][4], double* grad_pix,
                                    unsigned long long* queue, const LaunchShape& shape,
                                    int32_t grid, hipStream_t stream) {
    return reverse_launch<true>(c, dl_dI, nullptr, nullptr, count, c.n_pix, 0, cap, tape, jac,
                                grad_pix, queue, shape, grid, stream);
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
        if (metric == KERR) return occupancy(vjp_count_kernel<KERR>);
        if (metric == EINASTO) return occupancy(vjp_count_kernel<EINASTO>);
        return occupancy(vjp_count_kernel<CNFW>);
    }
    if (pass == 1) {
        if (metric == KERR) return occupancy(vjp_tape_kernel<KERR>);
        if (metric == EINASTO) return occupancy(vjp_tape_kernel<EINASTO>);
        return occupancy(vjp_tape_kernel<CNFW>);
    }
    if (pass == 3) {
        if (metric == KERR) return occupancy(vjp_tape_dense_kernel<KERR>);
        if (metric == EINASTO) return occupancy(vjp_tape_dense_kernel<EINASTO>);
        return occupancy(vjp_tape_dense_kernel<CNFW>);
    }
    if (metric == KERR) return occupancy(vjp_reverse_kernel<KERR, true>);
    if (metric == EINASTO) return occupancy(vjp_reverse_kernel<EINASTO, true>);
    return occupancy(vjp_reverse_kernel<CNFW, true>);
}

}  // namespace rt
