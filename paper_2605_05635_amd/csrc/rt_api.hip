// rt_api.hip -- the C ABI (include/rt.h): argument validation, per-image
// setup on the host (outer horizon, observer tetrad, screen, stop radii) and
// the stream-ordered launches of the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "rt.h"
#include "rt_device.h"
#include "rt_kernels.h"
#include "rt_points.h"
#include "rt_scan.h"

namespace {

thread_local std::string g_last_error;
thread_local hipEvent_t g_timing_start = nullptr, g_timing_stop = nullptr;
thread_local hipEvent_t g_timing_split = nullptr;   // after each mixed image's binary32 pass
thread_local rt_launch_config g_launch = {0, 0, 0, 0, 0};

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(RT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Images per batched launch: their constants must fit in the kernel's LDS
// table (~270 bytes each); larger batches run as consecutive launches.
constexpr int kMaxBatch = 128;
constexpr int kDefaultChunk = 64;
constexpr int32_t kDefaultTile = 8;   // ring-out hand-out: 8 x 8 pixel tiles
// Mixed precision: the binary32 bulk integrates at tolerances no tighter than
// kTol32Floor (binary32 stage values carry ~6e-8 relative rounding), and a ray
// continues in binary64 below kZoneFactor R_+.
constexpr double kTol32Floor = 1e-6;
constexpr double kZoneFactor = 1.5;

// Pinned host staging for the batched kernel's image tables, reused across
// calls on this thread; `ready` is recorded after the copy that reads it.
struct Staging {
    void* ptr = nullptr;
    size_t cap = 0;
    hipEvent_t ready = nullptr;
};
thread_local Staging g_staging;

int staging_reserve(size_t bytes, void** out) {
    Staging& s = g_staging;
    if (s.ready) {
        const hipError_t e = hipEventSynchronize(s.ready);   // previous copy has read it
        if (e != hipSuccess) return fail(RT_ERR_HIP, "staging event: %s", hipGetErrorString(e));
    } else if (hipEventCreateWithFlags(&s.ready, hipEventDisableTiming) != hipSuccess) {
        s.ready = nullptr;
        return fail(RT_ERR_HIP, "hipEventCreate failed");
    }
    if (s.cap < bytes) {
        if (s.ptr) (void)hipHostFree(s.ptr);
        s.ptr = nullptr;
        s.cap = 0;
        if (hipHostMalloc(&s.ptr, bytes, hipHostMallocDefault) != hipSuccess || !s.ptr) {
            (void)hipGetLastError();
            s.ptr = nullptr;
            return fail(RT_ERR_ALLOC, "pinned staging allocation of %zu bytes failed", bytes);
        }
        s.cap = bytes;
    }
    *out = s.ptr;
    return RT_OK;
}

rt::LaunchShape shape_for(int32_t nx, int32_t ny) {
    rt::LaunchShape sh;
    sh.chunk = g_launch.chunk > 0 ? g_launch.chunk : kDefaultChunk;
    if (g_launch.tile_w > 0 && g_launch.tile_h > 0) {
        sh.tile_w = g_launch.tile_w < nx ? g_launch.tile_w : nx;
        sh.tile_h = g_launch.tile_h < ny ? g_launch.tile_h : ny;
    } else {
        sh.tile_w = nx;
        sh.tile_h = 1;
    }
    return sh;
}

// Screen radius of the photon ring, for the hand-out order: the critical
// impact parameter min_r r / sqrt(1 - F(r)/r^2) of the non-rotating metric
// with the image's halo (sqrt(27) for Kerr), by a coarse scan (the order needs
// no precision).
double ring_radius(const rt::ImageConst& c) {
    double best = 1e300;
    for (int i = 0; i <= 2900; ++i) {
        const double r = 1.0 + 0.01 * i;
        double F, dF;
        rt::mass_function_any(c, r, F, dF);
        const double f = 1.0 - F / (r * r);
        if (f > 0.0) best = std::min(best, r / std::sqrt(f));
    }
    return best < 1e300 ? best : 0.0;
}

// Tiles of a screen in ring-out order: by the distance of the tile's centre
// from the photon ring's screen radius (ring_radius, centred on the screen
// origin, the direction of the hole), ties by tile index.  The rays near the
// ring, the longest, are handed out first; the shortest -- deep inside the
// shadow and far out -- fill the end of the launch, where the persistent
// grid drains.  One device table per screen, tile shape and halo, built on
// first use and kept (per thread).
struct TileOrder {
    int dev;
    int32_t nx, ny, tw, th, metric;
    double x0, dx, y0, dy, inv_lam, lam_c, eta_lc;
    int32_t* table;
};
thread_local std::vector<TileOrder> g_tile_orders;
constexpr size_t kMaxTileOrders = 64;

int tile_order(const rt::ImageConst& c, int32_t tw, int32_t th, const int32_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (const TileOrder& t : g_tile_orders)
        if (t.dev == dev && t.nx == c.nx && t.ny == c.ny && t.tw == tw && t.th == th &&
            t.x0 == c.x0 && t.dx == c.dx && t.y0 == c.y0 && t.dy == c.dy &&
            t.metric == c.metric && t.inv_lam == c.inv_lam && t.lam_c == c.lam_c &&
            t.eta_lc == c.eta_lc) {
            *out = t.table;
            return RT_OK;
        }
    if (g_tile_orders.size() >= kMaxTileOrders) {
        // earlier launches may still read the tables
        if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        for (TileOrder& t : g_tile_orders) (void)hipFree(t.table);
        g_tile_orders.clear();
    }
    const int32_t tiles_x = (c.nx + tw - 1) / tw, tiles_y = (c.ny + th - 1) / th;
    const int32_t n = tiles_x * tiles_y;
    const double ring = ring_radius(c);
    std::vector<int32_t> idx(n);
    std::vector<double> dist(n);
    for (int32_t i = 0; i < n; ++i) {
        idx[i] = i;
        const int32_t ty = i / tiles_x, tx = i - ty * tiles_x;
        const double w = std::min(tw, c.nx - tx * tw), h = std::min(th, c.ny - ty * th);
        const double X = c.x0 + (tx * tw + 0.5 * w) * c.dx;
        const double Y = c.y0 + (ty * th + 0.5 * h) * c.dy;
        dist[i] = std::fabs(std::sqrt(X * X + Y * Y) - ring);
    }
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int32_t a, int32_t b) { return dist[a] < dist[b]; });
    void* d = nullptr;
    if ((e = hipMalloc(&d, sizeof(int32_t) * n)) != hipSuccess || !d) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "tile order allocation failed");
    }
    if ((e = hipMemcpy(d, idx.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "tile order upload");
    }
    g_tile_orders.push_back(TileOrder{dev, c.nx, c.ny, tw, th, c.metric, c.x0, c.dx, c.y0, c.dy,
                                      c.inv_lam, c.lam_c, c.eta_lc, static_cast<int32_t*>(d)});
    *out = static_cast<int32_t*>(d);
    return RT_OK;
}

// The hand-out of one image's pixels under the current launch configuration.
int image_shape(const rt::ImageConst& c, rt::LaunchShape* sh) {
    if (g_launch.order == RT_ORDER_SCREEN) {
        *sh = shape_for(c.nx, c.ny);
        return RT_OK;
    }
    sh->chunk = g_launch.chunk > 0 ? g_launch.chunk : kDefaultChunk;
    sh->tile_w = std::min(g_launch.tile_w > 0 ? g_launch.tile_w : kDefaultTile, c.nx);
    sh->tile_h = std::min(g_launch.tile_h > 0 ? g_launch.tile_h : kDefaultTile, c.ny);
    return tile_order(c, sh->tile_w, sh->tile_h, &sh->order);
}

bool finite_all(std::initializer_list<double> v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

// Outer horizon: the largest root of Delta (eq. (33)) in (0.05, 50]
// (rt_scan.h).
// The horizon search walks Delta down from R = 50 in steps of 0.01 (about
// five thousand evaluations of the mass function, a few hundred microseconds
// of host time), so each thread keeps the results for its last kHorizonMemo
// spacetimes, keyed by every value Delta depends on (the same inputs give the
// same root: the memo changes no result, only the cost of a repeated call).
struct HorizonMemo {
    int32_t metric;
    double chi2, inv_lam, lam_c, inv_lam_c, eta_lc;
    bool found;
    double r_plus;
};
constexpr int kHorizonMemo = 128;   // a full batch of images
thread_local HorizonMemo g_horizon_memo[kHorizonMemo];
thread_local int g_horizon_used = 0, g_horizon_next = 0;

bool outer_horizon(const rt::ImageConst& c, double* r_plus) {
    for (int i = 0; i < g_horizon_used; ++i) {
        const HorizonMemo& m = g_horizon_memo[i];
        if (m.metric == c.metric && m.chi2 == c.chi2 && m.inv_lam == c.inv_lam &&
            m.lam_c == c.lam_c && m.inv_lam_c == c.inv_lam_c && m.eta_lc == c.eta_lc) {
            if (m.found) *r_plus = m.r_plus;
            return m.found;
        }
    }
    double r = 0.0;
    const bool found = rt::scan::largest_root(c, c.chi2, &r);
    g_horizon_memo[g_horizon_next] =
        HorizonMemo{c.metric, c.chi2, c.inv_lam, c.lam_c, c.inv_lam_c, c.eta_lc, found, r};
    g_horizon_next = (g_horizon_next + 1) % kHorizonMemo;
    if (g_horizon_used < kHorizonMemo) ++g_horizon_used;
    if (found) *r_plus = r;
    return found;
}

// Validates p and fills the image constants.  Returns RT_OK or an error code.
rt::Coeffs<double> coeffs_of(const rt::ImageConst& c) {
    return rt::Coeffs<double>{c.chi, c.chi2, c.inv_lam, c.lam_c, c.inv_lam_c, c.eta_lc};
}

void sin_cos(double th, double& s, double& co) {
    s = std::sin(th);
    co = std::cos(th);
}
template <int N>
void sin_cos(const rt::Dual<N>& th, rt::Dual<N>& s, rt::Dual<N>& co) {
    const double sv = std::sin(th.v), cv = std::cos(th.v);
    s = rt::chain(th, sv, cv);
    co = rt::chain(th, cv, -sv);
}

template <class S>
void mass_of(int metric, const rt::Coeffs<S>& k, const S& R, S& F, S& dF) {
    if (metric == rt::EINASTO)
        rt::mass_function<rt::EINASTO>(k, R, F, dF);
    else if (metric == rt::CNFW)
        rt::mass_function<rt::CNFW>(k, R, F, dF);
    else
        rt::mass_function<rt::KERR>(k, R, F, dF);
}

// The static observer's frame at (R_o, theta_o): the metric of eqs. (27)-(31)
// and the ZAMO lapse of eqs. (63)-(65).  out = {N_o, g_Tphi/sqrt(g_phiphi),
// sqrt(g_phiphi), sqrt(g_RR), sqrt(g_thth)}.  S is double, or a dual number
// for the derivatives of the screen map along the image parameters.
template <class S>
bool observer_frame(int metric, const rt::Coeffs<S>& k, const S& th, double R, S out[5]) {
    S F, dF;
    mass_of(metric, k, S(R), F, dF);
    S s, co;
    sin_cos(th, s, co);
    const S s2 = s * s;
    const S Sig = R * R + k.chi2 * co * co;
    const S Del = R * R - F + k.chi2;
    const S gTT = -(1.0 - F / Sig);
    const S gTp = -k.chi * F * s2 / Sig;
    const S gRR = Sig / Del;
    const S gthth = Sig;
    const S gpp = s2 * (R * R + k.chi2 + k.chi2 * F * s2 / Sig);
    const S N2 = gTp * gTp / gpp - gTT;  // -(g_TT + 2 w g_Tphi + w^2 g_phiphi), w = -g_Tphi/g_phiphi
    if (!(rt::value_of(Del) > 0.0) || !(rt::value_of(N2) > 0.0) || !(rt::value_of(gpp) > 0.0))
        return false;
    using std::sqrt;
    out[0] = sqrt(N2);
    out[2] = sqrt(gpp);
    out[1] = gTp / out[2];
    out[3] = sqrt(gRR);
    out[4] = sqrt(gthth);
    return true;
}

int setup_image(const rt_image_params* p, int index, bool emission, rt::ImageConst* c,
                double* r_plus_out) {
    if (!p) return fail(RT_ERR_ARG, "image %d: null parameter pointer", index);
    if (p->metric < RT_KERR || p->metric > RT_CNFW)
        return fail(RT_ERR_ARG, "image %d: unknown metric %d", index, p->metric);
    if (p->precision != RT_FP64 && p->precision != RT_MIXED)
        return fail(RT_ERR_ARG, "image %d: unsupported precision %d", index, p->precision);
    if (p->reserved != 0) return fail(RT_ERR_ARG, "image %d: reserved field must be 0", index);
    if (!finite_all({p->spin, p->halo[0], p->halo[1], p->incl, p->r_obs, p->x_min, p->x_max,
                     p->y_min, p->y_max, p->rtol, p->atol, p->r_stop_fac, p->r_esc_fac, p->r_in,
                     p->r_out, p->emis_pow, p->sigma_in, p->sigma_out, p->h0}))
        return fail(RT_ERR_ARG, "image %d: non-finite parameter", index);
    if (p->nx < 1 || p->ny < 1 || static_cast<int64_t>(p->nx) * p->ny >= (int64_t(1) << 31))
        return fail(RT_ERR_ARG, "image %d: bad screen size %d x %d", index, p->nx, p->ny);
    if (!(p->x_min < p->x_max) || !(p->y_min < p->y_max))
        return fail(RT_ERR_ARG, "image %d: empty screen extent", index);
    if (!(p->incl > 0.0) || !(p->incl < M_PI))
        return fail(RT_ERR_ARG, "image %d: inclination must lie in (0, pi)", index);
    if (!(p->rtol > 0.0) || !(p->atol > 0.0) || !(p->h0 > 0.0))
        return fail(RT_ERR_ARG, "image %d: rtol, atol and h0 must be positive", index);
    if (!(p->r_stop_fac > 1.0) || !(p->r_esc_fac > 1.0))
        return fail(RT_ERR_ARG, "image %d: stop factors must exceed 1", index);
    if (p->max_attempts < 1) return fail(RT_ERR_ARG, "image %d: max_attempts < 1", index);
    if (p->metric == RT_EINASTO && !(p->halo[0] > 0.0))
        return fail(RT_ERR_ARG, "image %d: Einasto lambda_E must be positive", index);
    if (p->metric == RT_CNFW && (!(p->halo[0] >= 0.0) || !(p->halo[1] > 0.0)))
        return fail(RT_ERR_ARG, "image %d: cored-NFW needs eta >= 0, lambda_c > 0", index);

    std::memset(c, 0, sizeof *c);
    c->metric = p->metric;
    c->max_attempts = p->max_attempts;
    c->nx = p->nx;
    c->ny = p->ny;
    c->n_pix = static_cast<int64_t>(p->nx) * p->ny;
    c->chi = p->spin;
    c->chi2 = p->spin * p->spin;
    if (p->metric == RT_EINASTO) c->inv_lam = 1.0 / p->halo[0];
    if (p->metric == RT_CNFW) {
        c->lam_c = p->halo[1];
        c->inv_lam_c = 1.0 / p->halo[1];
        c->eta_lc = p->halo[0] * p->halo[1];
        // exponent of eq. (13) = eta lambda_c P(R) in [-eta, 0] for eta >= 0: P(R) =
        // 1/(R + lambda_c) - (2/R) log(1 + R/lambda_c) increases from -1/lambda_c
        // (R -> 0) to 0
        c->ex_near = (p->halo[0] >= 0.0 && p->halo[0] <= rt::dm::kExpm1Near) ? 1 : 0;
    }
    double r_plus = 0.0;
    if (!outer_horizon(*c, &r_plus))
        return fail(RT_ERR_NO_HORIZON, "image %d: Delta(R) has no root in (0.05, 50]", index);
    if (r_plus_out) *r_plus_out = r_plus;
    c->r_stop = p->r_stop_fac * r_plus;
    c->r_esc = p->r_esc_fac * p->r_obs;
    c->r_zone = kZoneFactor * r_plus;
    c->rtol32 = std::max(p->rtol, kTol32Floor);
    c->atol32 = std::max(p->atol, kTol32Floor);
    c->r_in = p->r_in > 0.0 ? p->r_in : r_plus;
    c->r_out = p->r_out;
    if (!(c->r_out > c->r_in)) return fail(RT_ERR_ARG, "image %d: need r_out > r_in", index);
    if (!(p->r_obs > c->r_stop) || !(p->r_obs > c->r_out))
        return fail(RT_ERR_ARG, "image %d: observer must lie outside the disc and horizon", index);

    // Observer metric at (R_o, theta_o), eqs. (27)-(31), and the ZAMO (63)-(65).
    double frame[5];
    if (!observer_frame(c->metric, coeffs_of(*c), p->incl, p->r_obs, frame))
        return fail(RT_ERR_ARG, "image %d: no static observer frame at R_o", index);
    c->r_obs = p->r_obs;
    c->incl = p->incl;
    c->obs_N = frame[0];
    c->obs_gTph_over_sq_gphph = frame[1];
    c->obs_sq_gphph = frame[2];
    c->obs_sq_gRR = frame[3];
    c->obs_sq_gthth = frame[4];

    c->dx = (p->x_max - p->x_min) / p->nx;
    c->dy = (p->y_max - p->y_min) / p->ny;
    c->x0 = p->x_min;
    c->y0 = p->y_min;
    c->rtol = p->rtol;
    c->atol = p->atol;
    c->h0 = p->h0;
    c->emis_pow = p->emis_pow;
    c->sigma_in = p->sigma_in;
    c->sigma_out = p->sigma_out;
    c->taper = (p->sigma_in > 0.0 && p->sigma_out > 0.0) ? 1 : 0;
    c->inv_r_in = 1.0 / c->r_in;
    c->tin = c->taper ? 2.0 / p->sigma_in : 0.0;
    c->tout = c->taper ? 2.0 / p->sigma_out : 0.0;
    c->emission = emission ? 1 : 0;
    return RT_OK;
}

struct DeviceInfo {
    int cus = 0;
    int blocks_per_cu[3] = {0, 0, 0};
    int batch_blocks_per_cu = 0;   // at the largest batch table
};

int device_info(DeviceInfo* info) {
    static DeviceInfo cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(RT_ERR_HIP, "device index %d out of range", dev);
    DeviceInfo& d = cache[dev];
    if (d.cus == 0) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        for (int m = 0; m < 3; ++m) d.blocks_per_cu[m] = rt::max_blocks_per_cu(m);
        d.batch_blocks_per_cu = rt::max_batch_blocks_per_cu(kMaxBatch);
        d.cus = cus;
    }
    *info = d;
    return RT_OK;
}

template <class T>
int check_device_ptr(const T* ptr, const char* name, int index) {
    if (!ptr) return RT_OK;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RT_ERR_ARG, "image %d: %s is not device-accessible memory", index, name);
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(RT_ERR_ARG, "image %d: %s is not device memory", index, name);
    return RT_OK;
}

// Per-thread, per-device copy of the last mixed-precision call's counters
// (rays finished in binary64, of which traced again from the screen),
// written by the device at the end of each call.
thread_local long long* g_mixed_stats[64] = {};

int mixed_stats_buffer(long long** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(RT_ERR_HIP, "device index %d out of range", dev);
    if (!g_mixed_stats[dev]) {
        void* p = nullptr;
        if ((e = hipMalloc(&p, 4 * sizeof(long long))) != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(RT_ERR_ALLOC, "mixed-precision statistics buffer allocation failed");
        }
        const long long zeros[4] = {0, 0, 0, 0};
        if ((e = hipMemcpy(p, zeros, sizeof zeros, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "statistics buffer initialisation");
        g_mixed_stats[dev] = static_cast<long long*>(p);
    }
    *out = g_mixed_stats[dev];
    return RT_OK;
}

int trace_common(const rt_image_params* params, int32_t n_images, const rt_image_out* out,
                 void* hip_stream, bool emission) {
    g_last_error.clear();
    if (!params || !out) return fail(RT_ERR_ARG, "null params or out");
    if (n_images < 1) return fail(RT_ERR_ARG, "n_images must be >= 1");
    std::vector<rt::ImageConst> consts(n_images);
    for (int i = 0; i < n_images; ++i) {
        const int rc = setup_image(&params[i], i, emission, &consts[i], nullptr);
        if (rc != RT_OK) return rc;
        if (emission && out[i].reduce && !out[i].intensity)
            return fail(RT_ERR_ARG, "image %d: reduce needs the intensity output", i);
    }
    DeviceInfo info;
    int rc = device_info(&info);
    if (rc != RT_OK) return rc;
    for (int i = 0; i < n_images; ++i) {
        const rt_image_out& o = out[i];
        if ((rc = check_device_ptr(o.ncross, "ncross", i)) || (rc = check_device_ptr(o.status, "status", i)) ||
            (rc = check_device_ptr(o.r_em, "r_em", i)) || (rc = check_device_ptr(o.phi_em, "phi_em", i)) ||
            (rc = check_device_ptr(o.t_em, "t_em", i)) || (rc = check_device_ptr(o.g_em, "g_em", i)) ||
            (rc = check_device_ptr(o.intensity, "intensity", i)) ||
            (rc = check_device_ptr(o.intensity_n, "intensity_n", i)) ||
            (rc = check_device_ptr(o.attempts, "attempts", i)) ||
            (rc = check_device_ptr(o.reduce, "reduce", i)))
            return rc;
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::vector<rt::OutPtrs> optrs(n_images);
    for (int i = 0; i < n_images; ++i)
        optrs[i] = rt::OutPtrs{out[i].ncross, out[i].status, out[i].r_em, out[i].phi_em,
                               out[i].t_em, emission ? out[i].g_em : nullptr,
                               emission ? out[i].intensity : nullptr,
                               emission ? out[i].intensity_n : nullptr, out[i].attempts};
    // Binary64 images: one launch for a single image, else batches grouped by
    // metric (stable), at most kMaxBatch per launch.  Mixed-precision images
    // run one by one after them.
    std::vector<int> order, mixed;
    for (int i = 0; i < n_images; ++i)
        (params[i].precision == RT_MIXED ? mixed : order).push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return consts[a].metric < consts[b].metric; });
    const int nf = static_cast<int>(order.size());
    const int n_launch = nf <= 1 ? nf : (nf + kMaxBatch - 1) / kMaxBatch;

    // Scratch (stream-ordered): work-queue counters (one per binary64 launch,
    // then two per mixed image), the reduction partials, per batched launch its
    // image table, output table and chunk prefix sums, then per mixed image its
    // counters and the hand-off records.
    auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
    bool any_reduce = false;
    for (int i = 0; i < n_images; ++i) any_reduce |= emission && out[i].reduce != nullptr;
    const int n_queue = n_launch + 2 * static_cast<int>(mixed.size());
    const size_t queue_bytes = up256(sizeof(unsigned long long) * std::max(n_queue, 1));
    const size_t part_bytes = any_reduce ? up256(sizeof(double) * 3 * rt::kReduceBlocks) : 0;
    const size_t table_bytes =
        nf <= 1 ? 0
                : up256(sizeof(rt::ImageConst) * nf) + up256(sizeof(rt::OutPtrs) * nf) +
                      up256(sizeof(int64_t) * (nf + n_launch));
    size_t mixed_bytes = 0;
    for (int i : mixed)
        mixed_bytes += 256 + up256(rt::mixed_record_bytes() * static_cast<size_t>(consts[i].n_pix));
    // The pass after the trace (the emission, and the NaN transfer-map records
    // beyond each pixel's crossings, which the binary64 trace kernels leave to
    // it) runs whenever either is wanted.  It reads ncross, and with emission
    // r_em: images that do not return them get scratch ones.
    bool maps = false;
    for (int i = 0; i < n_images; ++i) maps = maps || out[i].r_em || out[i].phi_em || out[i].t_em;
    const bool after_pass = emission || maps;
    size_t emit_bytes = 0;
    for (int i = 0; i < n_images; ++i) {
        if (after_pass && !out[i].ncross) emit_bytes += up256(static_cast<size_t>(consts[i].n_pix));
        if (emission && !out[i].r_em)
            emit_bytes += up256(sizeof(double) * 3 * static_cast<size_t>(consts[i].n_pix));
    }
    const size_t scratch_bytes = queue_bytes + part_bytes + table_bytes + mixed_bytes + emit_bytes;
    void* scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, scratch_bytes, stream);
    if (e != hipSuccess || !scratch) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "stream-ordered allocation of %zu scratch bytes failed",
                    scratch_bytes);
    }
    char* base = static_cast<char*>(scratch);
    unsigned long long* queue = reinterpret_cast<unsigned long long*>(base);
    double* partials = reinterpret_cast<double*>(base + queue_bytes);
    char* tables = base + queue_bytes + part_bytes;
    char* mixed_area = tables + table_bytes;
    char* emit_area = mixed_area + mixed_bytes;
    auto bail = [&](int code) {
        (void)hipFreeAsync(scratch, stream);
        return code;
    };
    for (int i = 0; i < n_images; ++i) {
        if (after_pass && !optrs[i].ncross) {
            optrs[i].ncross = reinterpret_cast<uint8_t*>(emit_area);
            emit_area += up256(static_cast<size_t>(consts[i].n_pix));
        }
        if (emission && !optrs[i].r_em) {
            optrs[i].r_em = reinterpret_cast<double*>(emit_area);
            emit_area += up256(sizeof(double) * 3 * static_cast<size_t>(consts[i].n_pix));
        }
    }

    rt::ImageConst* d_table = nullptr;
    rt::OutPtrs* d_outs = nullptr;
    int64_t* d_cs = nullptr;
    if (nf > 1) {
        const size_t tb = up256(sizeof(rt::ImageConst) * nf);
        const size_t ob = up256(sizeof(rt::OutPtrs) * nf);
        d_table = reinterpret_cast<rt::ImageConst*>(tables);
        d_outs = reinterpret_cast<rt::OutPtrs*>(tables + tb);
        d_cs = reinterpret_cast<int64_t*>(tables + tb + ob);
        void* host = nullptr;
        const int src = staging_reserve(table_bytes, &host);
        if (src != RT_OK) return bail(src);
        char* h = static_cast<char*>(host);
        auto* h_table = reinterpret_cast<rt::ImageConst*>(h);
        auto* h_outs = reinterpret_cast<rt::OutPtrs*>(h + tb);
        auto* h_cs = reinterpret_cast<int64_t*>(h + tb + ob);
        const rt::LaunchShape sh0 = shape_for(1, 1);
        for (int l = 0, pos = 0; l < n_launch; ++l) {
            const int lo = l * kMaxBatch, hi = std::min(nf, lo + kMaxBatch);
            int64_t acc = 0;
            for (int j = lo; j < hi; ++j) {
                h_table[j] = consts[order[j]];
                h_outs[j] = optrs[order[j]];
                h_cs[pos++] = acc;
                acc += (consts[order[j]].n_pix + sh0.chunk - 1) / sh0.chunk;
            }
            h_cs[pos++] = acc;
        }
        e = hipMemcpyAsync(tables, host, table_bytes, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipEventRecord(g_staging.ready, stream);
        if (e != hipSuccess) return bail(hip_fail(e, "image table upload"));
    }
    e = rt::launch_zero(queue, std::max(n_queue, 1), stream);
    if (e != hipSuccess) return bail(hip_fail(e, "queue reset launch"));
    if (g_timing_start) (void)hipEventRecord(g_timing_start, stream);
    auto grid_for = [&](int64_t pix, int per_cu) {
        const int64_t want_blocks = (pix + 255) / 256;
        if (g_launch.blocks_per_cu > 0 && g_launch.blocks_per_cu < per_cu)
            per_cu = g_launch.blocks_per_cu;
        const int64_t resident = static_cast<int64_t>(info.cus) * per_cu;
        return static_cast<int32_t>(std::max<int64_t>(1, std::min(want_blocks, resident)));
    };
    if (nf == 1) {
        const rt::ImageConst& c = consts[order[0]];
        rt::LaunchShape sh;
        if ((rc = image_shape(c, &sh)) != RT_OK) return bail(rc);
        e = rt::launch_trace(c, optrs[order[0]], queue, sh,
                             grid_for(c.n_pix, info.blocks_per_cu[c.metric]), stream);
        if (e != hipSuccess) return bail(hip_fail(e, "trace kernel launch"));
    } else {
        for (int l = 0, pos = 0; l < n_launch; ++l) {
            const int lo = l * kMaxBatch, hi = std::min(nf, lo + kMaxBatch);
            int64_t pix = 0;
            for (int j = lo; j < hi; ++j) pix += consts[order[j]].n_pix;
            e = rt::launch_trace_batch(d_table + lo, d_outs + lo, d_cs + pos, hi - lo, queue + l,
                                       shape_for(1, 1), grid_for(pix, info.batch_blocks_per_cu),
                                       stream);
            if (e != hipSuccess) return bail(hip_fail(e, "batched trace kernel launch"));
            pos += hi - lo + 1;
        }
    }
    long long* stats = nullptr;
    if (!mixed.empty() && (rc = mixed_stats_buffer(&stats)) != RT_OK) return bail(rc);
    for (size_t m = 0; m < mixed.size(); ++m) {
        const int i = mixed[m];
        const rt::ImageConst& c = consts[i];
        unsigned long long* q = queue + n_launch + 2 * m;
        rt::LaunchShape sh;
        if ((rc = image_shape(c, &sh)) != RT_OK) return bail(rc);
        unsigned int* counters = reinterpret_cast<unsigned int*>(mixed_area);
        double* records = reinterpret_cast<double*>(mixed_area + 256);
        mixed_area += 256 + up256(rt::mixed_record_bytes() * static_cast<size_t>(c.n_pix));
        if ((e = rt::launch_zero(reinterpret_cast<unsigned long long*>(counters), 32, stream)) !=
                hipSuccess ||
            (e = rt::launch_trace32(c, optrs[i], q, sh,
                                    grid_for(c.n_pix, rt::mixed_blocks_per_cu(c.metric, 0)),
                                    records, counters, stream)) != hipSuccess ||
            (g_timing_split && (e = hipEventRecord(g_timing_split, stream)) != hipSuccess) ||
            (e = rt::launch_resume(c, optrs[i], records, counters, q + 1, 16,
                                   grid_for(c.n_pix, rt::mixed_blocks_per_cu(c.metric, 1)),
                                   stream)) != hipSuccess ||
            (e = rt::launch_copy_counters(counters, stats, stream)) != hipSuccess)
            return bail(hip_fail(e, "mixed-precision kernel launch"));
    }
    if (g_timing_stop) (void)hipEventRecord(g_timing_stop, stream);
    if (after_pass) {
        e = hipSuccess;
        if (nf == 1) {
            e = rt::launch_emission(consts[order[0]], optrs[order[0]], stream);
        } else if (nf > 1) {
            for (int l = 0; l < n_launch && e == hipSuccess; ++l) {
                const int lo = l * kMaxBatch, hi = std::min(nf, lo + kMaxBatch);
                int64_t max_pix = 0;
                for (int j = lo; j < hi; ++j) max_pix = std::max(max_pix, consts[order[j]].n_pix);
                e = rt::launch_emission_batch(d_table + lo, d_outs + lo, hi - lo, max_pix, stream);
            }
        }
        // (the mixed-precision kernels write their own NaN records)
        for (size_t m = 0; m < mixed.size() && emission && e == hipSuccess; ++m)
            e = rt::launch_emission(consts[mixed[m]], optrs[mixed[m]], stream);
        if (e != hipSuccess) return bail(hip_fail(e, "emission kernel launch"));
    }
    for (int i = 0; i < n_images; ++i) {
        if (emission && out[i].reduce) {
            e = rt::launch_reduce(consts[i], out[i].intensity, partials, out[i].reduce, stream);
            if (e != hipSuccess) return bail(hip_fail(e, "reduce kernel launch"));
        }
    }
    e = hipFreeAsync(scratch, stream);
    if (e != hipSuccess) return hip_fail(e, "hipFreeAsync");
    return RT_OK;
}


// ------------------------------------------------------------ image gradient
thread_local int64_t g_ckpt_budget = int64_t(16) << 30;

// Per-thread, per-device copy of the last gradient's counters (rays reversed,
// steps reversed, recomputations that diverged), written by the device at the
// end of each call.
thread_local long long* g_vjp_stats_dev[64] = {};
thread_local int64_t g_vjp_slots = 0, g_vjp_bytes = 0;

// jac[m][j]: derivative of per-ray parameter m (the kernel's order: chi, three
// mass constants, window inner edge, five observer-frame constants,
// inclination) along q_j = (spin, incl, halo[0], halo[1]), or along
// (spin, incl, rho_s, r_s) for the density basis of the cored NFW halo, where
// eta = 4 pi rho_s r_s^2 and lambda_c = r_s.
int vjp_jacobian(const rt_image_params* p, const rt::ImageConst& c, double r_plus, int32_t basis,
                 double jac[rt::kVjpPrims][4]) {
    using D = rt::Dual<4>;
    rt::Coeffs<D> k{};
    k.chi = D::var(p->spin, 0);
    k.chi2 = k.chi * k.chi;
    const D th = D::var(p->incl, 1);
    const D h0 = D::var(p->halo[0], 2), h1 = D::var(p->halo[1], 3);
    if (c.metric == rt::EINASTO) k.inv_lam = 1.0 / h0;
    if (c.metric == rt::CNFW) {
        k.lam_c = h1;
        k.inv_lam_c = 1.0 / h1;
        k.eta_lc = h0 * h1;
    }
    D frame[5];
    if (!observer_frame(c.metric, k, th, p->r_obs, frame))
        return fail(RT_ERR_ARG, "no static observer frame at R_o");
    const D zero(0.0);
    const D* rows[rt::kVjpPrims] = {&k.chi, &zero, &zero, &zero, &zero,
                                    &frame[0], &frame[1], &frame[2], &frame[3], &frame[4], &th};
    if (c.metric == rt::EINASTO) rows[1] = &k.inv_lam;
    if (c.metric == rt::CNFW) {
        rows[1] = &k.lam_c;
        rows[2] = &k.inv_lam_c;
        rows[3] = &k.eta_lc;
    }
    for (int m = 0; m < rt::kVjpPrims; ++m)
        for (int j = 0; j < 4; ++j) jac[m][j] = rows[m]->d[j];
    // The window's inner edge is the outer horizon unless given: Delta(R_+) = 0
    // moves by dR_+ = -(dDelta/dq) / (dDelta/dR) (implicit function theorem).
    for (int j = 0; j < 4; ++j) jac[4][j] = 0.0;
    if (!(p->r_in > 0.0)) {
        D F, dF;
        mass_of(c.metric, k, D(r_plus), F, dF);
        const D Del = r_plus * r_plus - F + k.chi2;
        const double dDel_dR = 2.0 * r_plus - dF.v;
        for (int j = 0; j < 4; ++j) jac[4][j] = -Del.d[j] / dDel_dR;
    }
    if (basis == RT_GRAD_DENSITY) {
        const double eta = p->halo[0], lc = p->halo[1];
        for (int m = 0; m < rt::kVjpPrims; ++m) {
            const double d_eta = jac[m][2], d_lc = jac[m][3];
            jac[m][2] = d_eta * 4.0 * M_PI * lc * lc;
            jac[m][3] = d_lc + d_eta * 2.0 * eta / lc;
        }
    }
    return RT_OK;
}

// Device counters of the gradient statistics (4 long longs per device).
int vjp_stats_buffer(long long** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(RT_ERR_HIP, "device index %d out of range", dev);
    if (!g_vjp_stats_dev[dev]) {
        void* p = nullptr;
        if ((e = hipMalloc(&p, 4 * sizeof(long long))) != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(RT_ERR_ALLOC, "gradient statistics buffer allocation failed");
        }
        const long long zeros[4] = {0, 0, 0, 0};
        if ((e = hipMemcpy(p, zeros, sizeof zeros, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "statistics buffer initialisation");
        g_vjp_stats_dev[dev] = static_cast<long long*>(p);
    }
    *out = g_vjp_stats_dev[dev];
    return RT_OK;
}

// Checkpoint slots per pixel for a screen of n_pix pixels within the budget:
// the most of kMaxSlots that fit, at least kMinSlots, even.
constexpr int64_t kMaxSlots = 32, kMinSlots = 4;
int32_t checkpoint_slots(int64_t n_pix) {
    const int64_t per = static_cast<int64_t>(sizeof(double)) * rt::kVjpCkptDoubles;
    int64_t s = g_ckpt_budget / (n_pix * per);
    s = std::max<int64_t>(kMinSlots, std::min<int64_t>(kMaxSlots, s));
    return static_cast<int32_t>(s & ~int64_t(1));
}

int image_vjp(const rt_image_params* params, const double* dl_dI, int32_t basis, double* grad,
              double* grad_pix, void* hip_stream) {
    g_last_error.clear();
    if (!params || !dl_dI || !grad) return fail(RT_ERR_ARG, "null params, dl_dI or grad");
    if (basis != RT_GRAD_NATIVE && basis != RT_GRAD_DENSITY)
        return fail(RT_ERR_ARG, "unknown gradient basis %d", basis);
    if (basis == RT_GRAD_DENSITY && params->metric != RT_CNFW)
        return fail(RT_ERR_ARG, "the density basis applies to the cored-NFW metric only");
    if (params->precision != RT_FP64)
        return fail(RT_ERR_ARG, "the gradient is taken of the binary64 trace (precision RT_FP64)");
    rt::ImageConst c;
    double r_plus = 0.0;
    int rc = setup_image(params, 0, true, &c, &r_plus);
    if (rc != RT_OK) return rc;
    double jac[rt::kVjpPrims][4];
    if ((rc = vjp_jacobian(params, c, r_plus, basis, jac)) != RT_OK) return rc;
    if ((rc = check_device_ptr(dl_dI, "dl_dI", 0)) || (rc = check_device_ptr(grad, "grad", 0)) ||
        (rc = check_device_ptr(grad_pix, "grad_pix", 0)))
        return rc;
    DeviceInfo info;
    if ((rc = device_info(&info)) != RT_OK) return rc;
    long long* stats = nullptr;
    if ((rc = vjp_stats_buffer(&stats)) != RT_OK) return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int64_t n_pix = c.n_pix;
    auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
    auto grid_of = [&](int pass, int64_t items) {
        const int64_t want = (items + rt::kBlock - 1) / rt::kBlock;
        int per_cu = rt::vjp_blocks_per_cu(c.metric, pass);
        if (g_launch.blocks_per_cu > 0 && g_launch.blocks_per_cu < per_cu)
            per_cu = g_launch.blocks_per_cu;
        const int64_t resident = static_cast<int64_t>(info.cus) * per_cu;
        return static_cast<int32_t>(std::max<int64_t>(1, std::min(want, resident)));
    };
    const int32_t slots = checkpoint_slots(n_pix);
    const int32_t grid_fwd = grid_of(0, n_pix), grid_bwd = grid_of(1, n_pix);

    // Scratch (stream-ordered, released at the end of the call): queue
    // counters, gradient counters, count and interval per pixel, the
    // checkpoints, the backward lanes' step buffers, gradient partials and the
    // per-pixel gradients when the caller passes none.
    const size_t q_bytes = 512;
    const size_t cnt_bytes = up256(sizeof(int32_t) * n_pix);
    const size_t ck_bytes =
        up256(sizeof(double) * rt::kVjpCkptDoubles * static_cast<size_t>(slots) * n_pix);
    const size_t buf_bytes = up256(static_cast<size_t>(rt::kVjpRecBytes) * rt::kVjpBuf *
                                   static_cast<size_t>(grid_bwd) * rt::kBlock);
    const size_t part_bytes = up256(sizeof(double) * 4 * rt::kGradBlocks);
    const size_t gp_bytes = grad_pix ? 0 : up256(sizeof(double) * 4 * n_pix);
    const size_t total = q_bytes + 2 * cnt_bytes + ck_bytes + buf_bytes + part_bytes + gp_bytes;
    void* scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, total, stream);
    if (e != hipSuccess || !scratch) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "stream-ordered allocation of %zu gradient bytes failed", total);
    }
    char* base = static_cast<char*>(scratch);
    unsigned long long* queue = reinterpret_cast<unsigned long long*>(base);
    unsigned long long* counters = reinterpret_cast<unsigned long long*>(base + 256);
    int32_t* count = reinterpret_cast<int32_t*>(base + q_bytes);
    int32_t* kseg = reinterpret_cast<int32_t*>(base + q_bytes + cnt_bytes);
    double* ckpt = reinterpret_cast<double*>(base + q_bytes + 2 * cnt_bytes);
    double* lane_buf = reinterpret_cast<double*>(base + q_bytes + 2 * cnt_bytes + ck_bytes);
    double* partials =
        reinterpret_cast<double*>(base + q_bytes + 2 * cnt_bytes + ck_bytes + buf_bytes);
    double* gp = grad_pix ? grad_pix
                          : reinterpret_cast<double*>(base + q_bytes + 2 * cnt_bytes + ck_bytes +
                                                      buf_bytes + part_bytes);
    auto bail = [&](int code) {
        (void)hipFreeAsync(scratch, stream);
        return code;
    };
    rt::LaunchShape shape;
    if ((rc = image_shape(c, &shape)) != RT_OK) return bail(rc);
    if ((e = rt::launch_zero(queue, 64, stream)) != hipSuccess)
        return bail(hip_fail(e, "queue reset launch"));
    if ((e = rt::launch_fill_zero(gp, 4 * n_pix, stream)) != hipSuccess)
        return bail(hip_fail(e, "gradient fill launch"));
    if ((e = rt::launch_vjp_forward(c, dl_dI, slots, ckpt, count, kseg, counters, queue, shape,
                                    grid_fwd, stream)) != hipSuccess)
        return bail(hip_fail(e, "forward checkpoint kernel launch"));
    if ((e = rt::launch_vjp_backward(c, dl_dI, count, kseg, slots, ckpt, lane_buf, jac, gp,
                                     counters, queue + 1, shape, grid_bwd, stream)) != hipSuccess)
        return bail(hip_fail(e, "backward kernel launch"));
    if ((e = rt::launch_grad_reduce(gp, n_pix, partials, grad, stream)) != hipSuccess)
        return bail(hip_fail(e, "gradient reduction launch"));
    if ((e = rt::launch_copy_vjp_stats(counters, stats, stream)) != hipSuccess)
        return bail(hip_fail(e, "statistics copy launch"));
    g_vjp_slots = slots;
    g_vjp_bytes = static_cast<int64_t>(total);
    if ((e = hipFreeAsync(scratch, stream)) != hipSuccess) return hip_fail(e, "hipFreeAsync");
    return RT_OK;
}

// Arguments of the diagnostics entry points: validated, screen constants in c.
int diagnostics_args(const double* intensity, const rt_image_params* params, double bin_width,
                     int32_t n_bins, const double* out, const double* profile, rt::ImageConst* c) {
    if (!intensity || !params || !out) return fail(RT_ERR_ARG, "null intensity, params or out");
    if (n_bins < 1 || n_bins > (1 << 20)) return fail(RT_ERR_ARG, "n_bins must lie in [1, 2^20]");
    if (!std::isfinite(bin_width) || !(bin_width > 0.0))
        return fail(RT_ERR_ARG, "bin_width must be finite and positive");
    const rt_image_params* p = params;
    if (p->nx < 1 || p->ny < 1 || static_cast<int64_t>(p->nx) * p->ny >= (int64_t(1) << 31))
        return fail(RT_ERR_ARG, "bad screen size %d x %d", p->nx, p->ny);
    if (!finite_all({p->x_min, p->x_max, p->y_min, p->y_max}) || !(p->x_min < p->x_max) ||
        !(p->y_min < p->y_max))
        return fail(RT_ERR_ARG, "bad screen extent");
    std::memset(c, 0, sizeof *c);
    c->nx = p->nx;
    c->ny = p->ny;
    c->n_pix = static_cast<int64_t>(p->nx) * p->ny;
    c->x0 = p->x_min;
    c->dx = (p->x_max - p->x_min) / p->nx;
    c->y0 = p->y_min;
    c->dy = (p->y_max - p->y_min) / p->ny;
    int rc;
    if ((rc = check_device_ptr(intensity, "intensity", 0)) || (rc = check_device_ptr(out, "out", 0)) ||
        (rc = check_device_ptr(profile, "profile", 0)))
        return rc;
    return RT_OK;
}

int image_diagnostics(const double* intensity, const rt_image_params* params, double bin_width,
                      int32_t n_bins, double* out, double* profile, void* hip_stream) {
    rt::ImageConst c;
    int rc = diagnostics_args(intensity, params, bin_width, n_bins, out, profile, &c);
    if (rc != RT_OK) return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const size_t bytes = sizeof(double) * rt::diagnostics_scratch_doubles(n_bins);
    void* scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, bytes, stream);
    if (e != hipSuccess || !scratch) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "stream-ordered allocation of %zu scratch bytes failed", bytes);
    }
    e = rt::launch_diagnostics(c, intensity, bin_width, n_bins, out, profile,
                               static_cast<double*>(scratch), stream);
    const hipError_t ef = hipFreeAsync(scratch, stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics kernel launch");
    if (ef != hipSuccess) return hip_fail(ef, "hipFreeAsync");
    return RT_OK;
}

// As image_diagnostics, with the file-scope work array of rt_diagnostics.hip
// in place of stream-ordered scratch: no allocation of any kind.
int image_diagnostics_noalloc(const double* intensity, const rt_image_params* params,
                              double bin_width, int32_t n_bins, double* out, double* profile,
                              void* hip_stream) {
    rt::ImageConst c;
    int rc = diagnostics_args(intensity, params, bin_width, n_bins, out, profile, &c);
    if (rc != RT_OK) return rc;
    if (!profile && n_bins > rt::kNoAllocMaxBins)
        return fail(RT_ERR_ARG, "without a profile buffer n_bins may be at most %d",
                    rt::kNoAllocMaxBins);
    double* work = nullptr;
    size_t have = 0;
    hipError_t e = rt::diagnostics_static_work(&work, &have);
    if (e != hipSuccess) return hip_fail(e, "static work array lookup");
    if (rt::diagnostics_scratch_doubles(profile ? 0 : n_bins) > have)
        return fail(RT_ERR_ARG, "static work array too small");
    e = rt::launch_diagnostics(c, intensity, bin_width, n_bins, out, profile, work,
                               static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "diagnostics kernel launch");
    return RT_OK;
}

// Normalised visibility amplitudes of n images (rt_visibility_dft and its
// batch form): validation, the work layout, one stream-ordered scratch block
// (image table, flux partials, partial sums) and three kernel launches.
int visibility_images(const rt_vis_image* imgs, int32_t n, hipStream_t stream) {
    std::vector<rt::VisImage> tab(n);
    int32_t max_k = 0;
    for (int32_t i = 0; i < n; ++i) {
        const rt_vis_image& g = imgs[i];
        if (!g.intensity || !g.uv || (!g.amp && !g.vis))
            return fail(RT_ERR_ARG, "image %d: null intensity, uv or both outputs", i);
        if (g.reserved != 0) return fail(RT_ERR_ARG, "image %d: reserved field must be 0", i);
        if (g.K < 1 || g.K > (1 << 22)) return fail(RT_ERR_ARG, "image %d: K must lie in [1, 2^22]", i);
        if (g.nx < 1 || g.ny < 1 || static_cast<int64_t>(g.nx) * g.ny >= (int64_t(1) << 31))
            return fail(RT_ERR_ARG, "image %d: bad screen size %d x %d", i, g.nx, g.ny);
        if (!finite_all({g.x_min, g.x_max, g.y_min, g.y_max}) || !(g.x_min < g.x_max) ||
            !(g.y_min < g.y_max))
            return fail(RT_ERR_ARG, "image %d: bad screen extent", i);
        rt::VisImage& m = tab[i];
        std::memset(&m, 0, sizeof m);
        m.I = g.intensity;
        m.uv = g.uv;
        m.amp = g.amp;
        m.vis = g.vis;
        m.nx = g.nx;
        m.ny = g.ny;
        m.K = g.K;
        m.x0 = g.x_min;
        m.dx = (g.x_max - g.x_min) / g.nx;
        m.y0 = g.y_min;
        m.dy = (g.y_max - g.y_min) / g.ny;
        max_k = std::max(max_k, g.K);
    }
    for (int32_t i = 0; i < n; ++i) {
        const rt_vis_image& g = imgs[i];
        int rc;
        if ((rc = check_device_ptr(g.intensity, "intensity", i)) ||
            (rc = check_device_ptr(g.uv, "uv", i)) || (rc = check_device_ptr(g.amp, "amp", i)) ||
            (rc = check_device_ptr(g.vis, "vis", i)))
            return rc;
    }
    int64_t items = 0;
    for (const rt::VisImage& m : tab)
        items += static_cast<int64_t>((m.K + 63) / 64) * ((m.nx + rt::kVisCols - 1) / rt::kVisCols);
    if (items >= (int64_t(1) << 31)) return fail(RT_ERR_ARG, "too much visibility work for one call");
    int32_t n_items = 0;
    int64_t n_part = 0;
    rt::vis_layout(tab.data(), n, &n_items, &n_part);
    auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t tab_bytes = up256(sizeof(rt::VisImage) * n);
    const size_t flux_bytes = up256(sizeof(double) * rt::kVisFluxBlocks * n);
    const size_t part_bytes = up256(sizeof(double2) * static_cast<size_t>(n_part));
    void* mem = nullptr;
    hipError_t e = hipMallocAsync(&mem, tab_bytes + flux_bytes + part_bytes, stream);
    if (e != hipSuccess || !mem) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "stream-ordered allocation of %zu visibility bytes failed",
                    tab_bytes + flux_bytes + part_bytes);
    }
    char* base = static_cast<char*>(mem);
    auto bail = [&](int code) {
        (void)hipFreeAsync(mem, stream);
        return code;
    };
    void* host = nullptr;
    int rc = staging_reserve(sizeof(rt::VisImage) * n, &host);
    if (rc != RT_OK) return bail(rc);
    std::memcpy(host, tab.data(), sizeof(rt::VisImage) * n);
    if ((e = hipMemcpyAsync(base, host, sizeof(rt::VisImage) * n, hipMemcpyHostToDevice,
                            stream)) != hipSuccess ||
        (e = hipEventRecord(g_staging.ready, stream)) != hipSuccess)
        return bail(hip_fail(e, "visibility table upload"));
    e = rt::launch_visibility(reinterpret_cast<const rt::VisImage*>(base), n, n_items, max_k,
                              reinterpret_cast<double2*>(base + tab_bytes + flux_bytes),
                              reinterpret_cast<double*>(base + tab_bytes), stream);
    if (e != hipSuccess) return bail(hip_fail(e, "visibility kernel launch"));
    if ((e = hipFreeAsync(mem, stream)) != hipSuccess) return hip_fail(e, "hipFreeAsync");
    return RT_OK;
}

}  // namespace

extern "C" {

int rt_trace_image(const rt_image_params* params, int32_t n_images, const rt_image_out* out,
                   void* hip_stream) {
    return trace_common(params, n_images, out, hip_stream, true);
}

int rt_transfer_maps(const rt_image_params* params, int32_t n_images, const rt_image_out* out,
                     void* hip_stream) {
    return trace_common(params, n_images, out, hip_stream, false);
}

int rt_trace_thick(const rt_image_params* params, const rt_thick_disc* thick,
                   const rt_image_out* out, void* hip_stream) {
    g_last_error.clear();
    if (!params || !thick || !out) return fail(RT_ERR_ARG, "null params, thick or out");
    if (!finite_all({thick->r_scale, thick->h0, thick->h_slope}) || !(thick->r_scale > 0.0) ||
        !(thick->h0 > 0.0) || !(thick->h_slope >= 0.0))
        return fail(RT_ERR_ARG, "thick disc needs finite r_scale > 0, h0 > 0, h_slope >= 0");
    if (!out->intensity) return fail(RT_ERR_ARG, "the thick disc needs out->intensity");
    if (out->g_em || out->intensity_n || out->reduce)
        return fail(RT_ERR_ARG, "g_em, intensity_n and reduce are not produced by the thick disc");
    if (params->precision != RT_FP64)
        return fail(RT_ERR_ARG, "the thick disc is traced in binary64 (precision RT_FP64)");
    rt::ImageConst c;
    int rc = setup_image(params, 0, true, &c, nullptr);
    if (rc != RT_OK) return rc;
    c.thick_rs = thick->r_scale;
    c.inv_thick_rs = 1.0 / thick->r_scale;
    c.thick_h0 = thick->h0;
    c.thick_h = thick->h_slope;
    const rt_image_out& o = *out;
    if ((rc = check_device_ptr(o.ncross, "ncross", 0)) || (rc = check_device_ptr(o.status, "status", 0)) ||
        (rc = check_device_ptr(o.r_em, "r_em", 0)) || (rc = check_device_ptr(o.phi_em, "phi_em", 0)) ||
        (rc = check_device_ptr(o.t_em, "t_em", 0)) || (rc = check_device_ptr(o.intensity, "intensity", 0)) ||
        (rc = check_device_ptr(o.attempts, "attempts", 0)))
        return rc;
    const rt::OutPtrs optrs{o.ncross, o.status, o.r_em, o.phi_em, o.t_em, nullptr, o.intensity,
                            nullptr, o.attempts};
    DeviceInfo info;
    if ((rc = device_info(&info)) != RT_OK) return rc;
    rt::LaunchShape sh;
    if ((rc = image_shape(c, &sh)) != RT_OK) return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    void* q = nullptr;
    hipError_t e = hipMallocAsync(&q, 256, stream);
    if (e != hipSuccess || !q) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "stream-ordered allocation of the work queue failed");
    }
    auto* queue = static_cast<unsigned long long*>(q);
    const int64_t want = (c.n_pix + 255) / 256;
    const int64_t resident = static_cast<int64_t>(info.cus) * rt::thick_blocks_per_cu(c.metric);
    const int32_t grid = static_cast<int32_t>(std::max<int64_t>(1, std::min(want, resident)));
    e = rt::launch_zero(queue, 1, stream);
    if (e == hipSuccess) e = rt::launch_trace_thick(c, optrs, queue, sh, grid, stream);
    const hipError_t ef = hipFreeAsync(q, stream);
    if (e != hipSuccess) return hip_fail(e, "thick-disc kernel launch");
    if (ef != hipSuccess) return hip_fail(ef, "hipFreeAsync");
    return RT_OK;
}

int rt_parameter_scan(const rt_scan_point* points, int32_t n, double* out, void* hip_stream) {
    g_last_error.clear();
    if (!points || !out) return fail(RT_ERR_ARG, "null points or out");
    if (n < 1 || n > (1 << 24)) return fail(RT_ERR_ARG, "n must lie in [1, 2^24]");
    int rc;
    if ((rc = check_device_ptr(points, "points", 0)) || (rc = check_device_ptr(out, "out", 0)))
        return rc;
    const hipError_t e = rt::launch_scan(points, n, out, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "scan kernel launch");
    return RT_OK;
}

int rt_image_diagnostics(const double* intensity, const rt_image_params* params, double bin_width,
                         int32_t n_bins, double* out, double* profile, void* hip_stream) {
    g_last_error.clear();
    return image_diagnostics(intensity, params, bin_width, n_bins, out, profile, hip_stream);
}

int rt_relative_deviation(const double* q, const double* ref, int32_t n, double* delta,
                          void* hip_stream) {
    g_last_error.clear();
    if (!q || !ref || !delta) return fail(RT_ERR_ARG, "null q, ref or delta");
    if (n < 1 || n > (1 << 24)) return fail(RT_ERR_ARG, "n must lie in [1, 2^24]");
    int rc;
    if ((rc = check_device_ptr(q, "q", 0)) || (rc = check_device_ptr(ref, "ref", 0)) ||
        (rc = check_device_ptr(delta, "delta", 0)))
        return rc;
    const hipError_t e = rt::launch_relative(q, ref, n, delta, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "relative deviation kernel launch");
    return RT_OK;
}

int rt_image_diagnostics_noalloc(const double* intensity, const rt_image_params* params,
                                 double bin_width, int32_t n_bins, double* out, double* profile,
                                 void* hip_stream) {
    g_last_error.clear();
    return image_diagnostics_noalloc(intensity, params, bin_width, n_bins, out, profile,
                                     hip_stream);
}

int rt_trace_points(const rt_image_params* params, const double* xy, int64_t n,
                    const rt_image_out* out, void* hip_stream) {
    g_last_error.clear();
    if (!params || !xy || !out) return fail(RT_ERR_ARG, "null params, xy or out");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(RT_ERR_ARG, "n must lie in [1, 2^31)");
    if (params->precision != RT_FP64)
        return fail(RT_ERR_ARG, "screen points are traced in binary64 (precision RT_FP64)");
    const rt_image_out& o = *out;
    if (o.reduce) return fail(RT_ERR_ARG, "reduce is not produced for screen points");
    const bool emission = o.intensity || o.g_em || o.intensity_n;
    if (emission && (!o.ncross || !o.r_em))
        return fail(RT_ERR_ARG, "the emission of screen points needs out->ncross and out->r_em");
    rt::ImageConst c;
    int rc = setup_image(params, 0, emission, &c, nullptr);
    if (rc != RT_OK) return rc;
    c.n_pix = n;
    if ((rc = check_device_ptr(xy, "xy", 0)) || (rc = check_device_ptr(o.ncross, "ncross", 0)) ||
        (rc = check_device_ptr(o.status, "status", 0)) || (rc = check_device_ptr(o.r_em, "r_em", 0)) ||
        (rc = check_device_ptr(o.phi_em, "phi_em", 0)) || (rc = check_device_ptr(o.t_em, "t_em", 0)) ||
        (rc = check_device_ptr(o.g_em, "g_em", 0)) || (rc = check_device_ptr(o.intensity, "intensity", 0)) ||
        (rc = check_device_ptr(o.intensity_n, "intensity_n", 0)) ||
        (rc = check_device_ptr(o.attempts, "attempts", 0)))
        return rc;
    const rt::OutPtrs optrs{o.ncross, o.status, o.r_em, o.phi_em, o.t_em, o.g_em, o.intensity,
                            o.intensity_n, o.attempts};
    DeviceInfo info;
    if ((rc = device_info(&info)) != RT_OK) return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    void* q = nullptr;
    hipError_t e = hipMallocAsync(&q, 256, stream);
    if (e != hipSuccess || !q) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "stream-ordered allocation of the work queue failed");
    }
    auto* queue = static_cast<unsigned long long*>(q);
    const int64_t want = (n + 255) / 256;
    const int64_t resident = static_cast<int64_t>(info.cus) * rt::points_blocks_per_cu(c.metric);
    const int32_t grid = static_cast<int32_t>(std::max<int64_t>(1, std::min(want, resident)));
    e = rt::launch_zero(queue, 1, stream);
    if (e == hipSuccess) e = rt::launch_trace_points(c, xy, optrs, queue, grid, stream);
    const hipError_t ef = hipFreeAsync(q, stream);
    if (e != hipSuccess) return hip_fail(e, "screen-point kernel launch");
    if (ef != hipSuccess) return hip_fail(ef, "hipFreeAsync");
    return RT_OK;
}

int rt_refine_points(const rt_image_params* params, const uint8_t* ncross, const uint8_t* status,
                     int32_t sub, int64_t max_points, double* xy, int64_t* pix, int64_t* n_marked,
                     void* hip_stream) {
    g_last_error.clear();
    if (!params || !ncross || !status || !n_marked)
        return fail(RT_ERR_ARG, "null params, ncross, status or n_marked");
    if (sub < 1 || sub > 16) return fail(RT_ERR_ARG, "sub must lie in [1, 16]");
    if (max_points < 0) return fail(RT_ERR_ARG, "max_points must be >= 0");
    if (max_points > 0 && !xy) return fail(RT_ERR_ARG, "xy is null with max_points > 0");
    rt::ImageConst c;
    int rc = setup_image(params, 0, false, &c, nullptr);
    if (rc != RT_OK) return rc;
    if ((rc = check_device_ptr(ncross, "ncross", 0)) || (rc = check_device_ptr(status, "status", 0)) ||
        (rc = check_device_ptr(xy, "xy", 0)) || (rc = check_device_ptr(pix, "pix", 0)) ||
        (rc = check_device_ptr(n_marked, "n_marked", 0)))
        return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int64_t blocks = (c.n_pix + rt::kBlock - 1) / rt::kBlock;
    void* mem = nullptr;
    hipError_t e = hipMallocAsync(&mem, sizeof(int64_t) * static_cast<size_t>(blocks), stream);
    if (e != hipSuccess || !mem) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "stream-ordered allocation of the refinement counts failed");
    }
    const int64_t per_pixel = static_cast<int64_t>(sub) * sub;
    e = rt::launch_refine(c, ncross, status, sub, max_points / per_pixel, xy, pix, n_marked,
                          static_cast<int64_t*>(mem), stream);
    const hipError_t ef = hipFreeAsync(mem, stream);
    if (e != hipSuccess) return hip_fail(e, "refinement kernel launch");
    if (ef != hipSuccess) return hip_fail(ef, "hipFreeAsync");
    return RT_OK;
}

int rt_shadow_boundary(const rt_image_params* params, const double* dirs, int32_t n,
                       int32_t samples, double b_lo, double b_hi, double b_tol, double* out,
                       int32_t* status, int64_t* attempts, void* hip_stream) {
    g_last_error.clear();
    if (!params || !dirs || !out || !status) return fail(RT_ERR_ARG, "null params, dirs, out or status");
    if (n < 1 || n > (1 << 24)) return fail(RT_ERR_ARG, "n must lie in [1, 2^24]");
    if (samples != 16 && samples != 32 && samples != 64)
        return fail(RT_ERR_ARG, "samples must be 16, 32 or 64");
    if (!finite_all({b_lo, b_hi, b_tol}) || !(b_lo > 0.0) || !(b_lo < b_hi))
        return fail(RT_ERR_ARG, "need finite 0 < b_lo < b_hi");
    if (!(b_tol >= 1e-13 * b_hi))
        return fail(RT_ERR_ARG, "b_tol must be at least 1e-13 b_hi");
    if (params->precision != RT_FP64)
        return fail(RT_ERR_ARG, "the boundary search traces in binary64 (precision RT_FP64)");
    rt::ImageConst c;
    int rc = setup_image(params, 0, false, &c, nullptr);
    if (rc != RT_OK) return rc;
    if ((rc = check_device_ptr(dirs, "dirs", 0)) || (rc = check_device_ptr(out, "out", 0)) ||
        (rc = check_device_ptr(status, "status", 0)) ||
        (rc = check_device_ptr(attempts, "attempts", 0)))
        return rc;
    const hipError_t e = rt::launch_boundary(c, dirs, n, samples, b_lo, b_hi, b_tol, out, status, attempts,
                                             static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return hip_fail(e, "boundary kernel launch");
    return RT_OK;
}

int rt_shadow_boundary_samples(int32_t n) {
    g_last_error.clear();
    if (n < 1) return fail(RT_ERR_ARG, "n must be at least 1");
    DeviceInfo info;
    const int rc = device_info(&info);
    if (rc != RT_OK) return rc;
    const int64_t lanes = static_cast<int64_t>(info.cus) * 4 * 64;
    for (int s = 64; s > 16; s /= 2)
        if (static_cast<int64_t>(n) * s <= lanes) return s;
    return 16;
}

int rt_image_setup(const rt_image_params* params, double* setup) {
    g_last_error.clear();
    if (!setup) return fail(RT_ERR_ARG, "null setup pointer");
    rt::ImageConst c;
    double r_plus = 0.0;
    const int rc = setup_image(params, 0, true, &c, &r_plus);
    if (rc != RT_OK) return rc;
    setup[0] = r_plus;
    setup[1] = c.r_stop;
    setup[2] = c.r_esc;
    setup[3] = c.r_in;
    return RT_OK;
}

int rt_set_split_timing(void* event) {
    g_last_error.clear();
    g_timing_split = static_cast<hipEvent_t>(event);
    return RT_OK;
}

int rt_set_kernel_timing(void* start_event, void* stop_event) {
    g_last_error.clear();
    if ((start_event == nullptr) != (stop_event == nullptr))
        return fail(RT_ERR_ARG, "timing events must both be set or both be null");
    g_timing_start = static_cast<hipEvent_t>(start_event);
    g_timing_stop = static_cast<hipEvent_t>(stop_event);
    return RT_OK;
}

int rt_visibility_dft(const double* intensity, const rt_image_params* params, const double* uv,
                      int32_t K, double* amp, double* vis, void* hip_stream) {
    g_last_error.clear();
    if (!params) return fail(RT_ERR_ARG, "null params");
    const rt_vis_image img{intensity, uv, amp, vis, params->nx, params->ny, K, 0,
                           params->x_min, params->x_max, params->y_min, params->y_max};
    return visibility_images(&img, 1, static_cast<hipStream_t>(hip_stream));
}

int rt_visibility_dft_batch(const rt_vis_image* images, int32_t n_images, void* hip_stream) {
    g_last_error.clear();
    if (!images) return fail(RT_ERR_ARG, "null images");
    if (n_images < 1 || n_images > (1 << 16)) return fail(RT_ERR_ARG, "n_images must lie in [1, 2^16]");
    return visibility_images(images, n_images, static_cast<hipStream_t>(hip_stream));
}

int rt_visibility_rings(const double* intensity, const rt_image_params* params, const double* q,
                        int32_t n_q, int32_t n_angles, double* avg, double* cut,
                        void* hip_stream) {
    g_last_error.clear();
    if (!intensity || !params || !q || (!avg && !cut))
        return fail(RT_ERR_ARG, "null intensity, params, q or both outputs");
    if (n_q < 1 || n_angles < 1 || static_cast<int64_t>(n_q) * n_angles > (int64_t(1) << 22))
        return fail(RT_ERR_ARG, "need n_q >= 1, n_angles >= 1, n_q n_angles <= 2^22");
    int rc;
    if ((rc = check_device_ptr(q, "q", 0)) || (rc = check_device_ptr(avg, "avg", 0)) ||
        (rc = check_device_ptr(cut, "cut", 0)))
        return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int64_t n = static_cast<int64_t>(n_q) * n_angles;
    void* mem = nullptr;
    hipError_t e = hipMallocAsync(&mem, sizeof(double) * 3 * n, stream);
    if (e != hipSuccess || !mem) {
        (void)hipGetLastError();
        return fail(RT_ERR_ALLOC, "stream-ordered allocation of the ring points failed");
    }
    double* uv = static_cast<double*>(mem);
    double* amp = uv + 2 * n;
    auto bail = [&](int code) {
        (void)hipFreeAsync(mem, stream);
        return code;
    };
    if ((e = rt::launch_ring_points(q, n_q, n_angles, uv, stream)) != hipSuccess)
        return bail(hip_fail(e, "ring point kernel launch"));
    const rt_vis_image img{intensity, uv, amp, nullptr, params->nx, params->ny,
                           static_cast<int32_t>(n), 0, params->x_min, params->x_max,
                           params->y_min, params->y_max};
    if ((rc = visibility_images(&img, 1, stream)) != RT_OK) return bail(rc);
    if ((e = rt::launch_ring_average(amp, n_q, n_angles, avg, cut, stream)) != hipSuccess)
        return bail(hip_fail(e, "ring average kernel launch"));
    if ((e = hipFreeAsync(mem, stream)) != hipSuccess) return hip_fail(e, "hipFreeAsync");
    return RT_OK;
}

int rt_set_launch_config(const rt_launch_config* cfg) {
    g_last_error.clear();
    if (!cfg) {
        g_launch = rt_launch_config{0, 0, 0, 0, 0};
        return RT_OK;
    }
    if (cfg->chunk < 0 || cfg->chunk > 65536 || cfg->tile_w < 0 || cfg->tile_h < 0 ||
        (cfg->tile_w > 0) != (cfg->tile_h > 0) || cfg->blocks_per_cu < 0 ||
        cfg->blocks_per_cu > 64 || (cfg->order != RT_ORDER_CENTRE && cfg->order != RT_ORDER_SCREEN))
        return fail(RT_ERR_ARG, "launch config out of range");
    g_launch = *cfg;
    return RT_OK;
}

int rt_get_launch_config(rt_launch_config* cfg) {
    g_last_error.clear();
    if (!cfg) return fail(RT_ERR_ARG, "null launch config pointer");
    *cfg = g_launch;
    return RT_OK;
}

int rt_image_vjp(const rt_image_params* params, const double* dl_dI, int32_t basis,
                 double* grad, double* grad_pix, void* hip_stream) {
    return image_vjp(params, dl_dI, basis, grad, grad_pix, hip_stream);
}

int rt_mixed_stats(int64_t* out) {
    g_last_error.clear();
    if (!out) return fail(RT_ERR_ARG, "null stats pointer");
    long long* d = nullptr;
    int rc = mixed_stats_buffer(&d);
    if (rc != RT_OK) return rc;
    long long h[4] = {0, 0, 0, 0};
    const hipError_t e = hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "statistics read-back");
    for (int i = 0; i < 4; ++i) out[i] = h[i];
    return RT_OK;
}

int rt_set_checkpoint_budget(int64_t bytes) {
    g_last_error.clear();
    if (bytes < (int64_t(1) << 20)) return fail(RT_ERR_ARG, "checkpoint budget below 1 MiB");
    g_ckpt_budget = bytes;
    return RT_OK;
}

int rt_vjp_stats(int64_t* out) {
    g_last_error.clear();
    if (!out) return fail(RT_ERR_ARG, "null stats pointer");
    long long* d = nullptr;
    const int rc = vjp_stats_buffer(&d);
    if (rc != RT_OK) return rc;
    long long h[3] = {0, 0, 0};
    const hipError_t e = hipMemcpy(h, d, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "statistics read-back");
    out[0] = h[0];
    out[1] = h[1];
    out[2] = g_vjp_slots;
    out[3] = g_vjp_bytes;
    out[4] = h[2];
    return RT_OK;
}

const char* rt_last_error(void) { return g_last_error.c_str(); }

int rt_version(void) { return RT_VERSION; }

}  // extern "C"
