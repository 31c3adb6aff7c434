// C ABI of libxct.so: argument validation, per-geometry device tables and
// dispatch of the filter, back-projection, forward-projection and reduction
// kernels.  See include/xct.h for the contract of every entry point.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "xct_internal.h"

using namespace xct;

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return XCT_EHIP;
}

bool dtype_ok(int t) { return t == XCT_F32 || t == XCT_F16 || t == XCT_BF16; }
size_t dtype_size(int t) { return t == XCT_F32 ? 4 : 2; }

// ---------------------------------------------------------------- validation

int check_geometry(const xct_geometry *g, bool need_angles)
{
    if (!g) return XCT_EINVAL;
    if (g->n_angles <= 0 || g->n_det <= 0 || g->nx <= 0 || g->ny <= 0) return XCT_EINVAL;
    if (!std::isfinite(g->det_pitch) || !(g->det_pitch > 0)) return XCT_EINVAL;
    if (!std::isfinite(g->pixel_size) || !(g->pixel_size > 0)) return XCT_EINVAL;
    if (!std::isfinite(g->center)) return XCT_EINVAL;
    if (need_angles) {
        if (!g->angles) return XCT_EINVAL;
        for (int k = 0; k < g->n_angles; ++k)
            if (!std::isfinite(g->angles[k])) return XCT_EINVAL;
    }
    if (g->n_det > 65536 || g->nx > 65536 || g->ny > 65536 || g->n_angles > (1 << 20))
        return XCT_ETOOBIG;
    const double ratio = g->pixel_size / g->det_pitch;
    if (ratio > 16.0 || ratio < 1.0 / 16.0) return XCT_ETOOBIG;
    if (std::fabs(g->center) > 1e6) return XCT_ETOOBIG;
    return XCT_OK;
}

int check_slices(const xct_geometry *g, int32_t n_slices)
{
    if (n_slices <= 0) return XCT_EINVAL;
    const double lim = 4.0e18;
    if ((double)n_slices * g->n_angles * g->n_det > lim) return XCT_ETOOBIG;
    if ((double)n_slices * g->nx * g->ny > lim) return XCT_ETOOBIG;
    return XCT_OK;
}

// ---------------------------------------------------------------- device tables

struct GeoTables {
    float2 *cs = nullptr;
    double2 *csd = nullptr;
};

struct FilterTables {
    float2 *tw = nullptr;
    float *H = nullptr;
};

struct FPTables {
    FPAngle *ang = nullptr;
    FPBlock *blocks = nullptr;
    int n_blocks = 0;
    int rows[2] = {0, 0}, pitch[2] = {0, 0};  // staging shape for 1 and 4 slices per workgroup
};

std::mutex g_mu;
std::unordered_map<std::string, GeoTables> g_geo;
std::unordered_map<std::string, FilterTables> g_filt;
std::unordered_map<std::string, FPTables> g_fp;
std::unordered_map<std::string, float *> g_blur;
std::unordered_map<std::string, float *> g_offset;

template <typename T>
void key_append(std::string &k, const T &v)
{
    k.append(reinterpret_cast<const char *>(&v), sizeof(T));
}

int current_device(int *dev)
{
    hipError_t e = hipGetDevice(dev);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

// cos/sin of every angle times pixel/pitch, in FP32 (inner loops) and FP64
// (window anchors), rounded once from FP64 host trigonometry.
int geo_tables(const xct_geometry *g, GeoTables *out)
{
    int dev;
    if (int rc = current_device(&dev)) return rc;
    const double r = g->pixel_size / g->det_pitch;
    std::string key;
    key_append(key, dev);
    key_append(key, r);
    key.append(reinterpret_cast<const char *>(g->angles), sizeof(double) * g->n_angles);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_geo.find(key);
    if (it != g_geo.end()) {
        *out = it->second;
        return XCT_OK;
    }
    const int n = g->n_angles;
    std::vector<float2> cs(n);
    std::vector<double2> csd(n);
    for (int k = 0; k < n; ++k) {
        const double c = std::cos(g->angles[k]) * r, s = std::sin(g->angles[k]) * r;
        csd[k] = make_double2(c, s);
        cs[k] = make_float2((float)c, (float)s);
    }
    GeoTables t;
    hipError_t e = hipMalloc(&t.cs, sizeof(float2) * n);
    if (e == hipSuccess) e = hipMalloc(&t.csd, sizeof(double2) * n);
    if (e == hipSuccess) e = hipMemcpy(t.cs, cs.data(), sizeof(float2) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.csd, csd.data(), sizeof(double2) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (t.cs) (void)hipFree(t.cs);
        if (t.csd) (void)hipFree(t.csd);
        return hip_fail(e);
    }
    g_geo.emplace(key, t);
    *out = t;
    return XCT_OK;
}

// Unit-sum sampled Gaussian of standard deviation sigma over -R..R,
// R = int(4 sigma + 0.5), in FP64 rounded once to FP32, cached on the device.
int blur_taps(float sigma, int radius, const float **out)
{
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::string key;
    key_append(key, dev);
    key_append(key, sigma);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_blur.find(key);
    if (it != g_blur.end()) {
        *out = it->second;
        return XCT_OK;
    }
    std::vector<double> g(2 * radius + 1);
    double sum = 0.0;
    for (int m = -radius; m <= radius; ++m) {
        const double t = (double)m / (double)sigma;
        g[m + radius] = std::exp(-0.5 * t * t);
        sum += g[m + radius];
    }
    std::vector<float> g32(g.size());
    for (size_t i = 0; i < g.size(); ++i) g32[i] = (float)(g[i] / sum);
    float *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(float) * g32.size());
    if (e == hipSuccess) e = hipMemcpy(d, g32.data(), sizeof(float) * g32.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return hip_fail(e);
    }
    g_blur.emplace(key, d);
    *out = d;
    return XCT_OK;
}

// Virtual detector of a full-turn scan: the physical bins and their mirror
// images about the axis (bin 2c - n), renumbered from 0.  `first` is the
// virtual bin of physical bin 0.  Needs 2c integral and the axis on the
// detector.
void offset_virtual(const xct_geometry *g, int *nv, double *cv, int *first)
{
    const int nc = g->n_det;
    const int two_c = (int)std::nearbyint(2.0 * g->center);
    if ((nc - 1) - g->center >= g->center) {  // longer side to the right of the axis
        const int lo = two_c - (nc - 1);
        *nv = nc - lo;
        *cv = g->center - lo;
        *first = -lo;
    } else {
        *nv = two_c + 1;
        *cv = g->center;
        *first = 0;
    }
}

// Redundancy weights of a full-turn scan (offset scan, Section V-A b): with
// t = (n - c) / overlap, positive on the detector's longer side,
// w = 0 (t <= -1), sin^2(pi (1 + t) / 4) (|t| < 1), 1 (t >= 1), so that the
// two measurements of every ray, bins n and 2c - n half a turn apart, weigh
// one together.  FP64 on the host, rounded once, cached on the device.
int offset_weights(const xct_geometry *g, double overlap, const float **out)
{
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::string key;
    key_append(key, dev);
    key_append(key, g->n_det);
    key_append(key, g->center);
    key_append(key, overlap);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_offset.find(key);
    if (it != g_offset.end()) {
        *out = it->second;
        return XCT_OK;
    }
    const int nc = g->n_det;
    const double side = ((nc - 1) - g->center >= g->center) ? 1.0 : -1.0;
    std::vector<float> w(nc);
    for (int n = 0; n < nc; ++n) {
        const double t = side * ((double)n - g->center) / overlap;
        double v = 1.0;
        if (t <= -1.0) v = 0.0;
        else if (t < 1.0) {
            const double sn = std::sin(0.25 * M_PI * (1.0 + t));
            v = sn * sn;
        }
        w[n] = (float)v;
    }
    float *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(float) * nc);
    if (e == hipSuccess) e = hipMemcpy(d, w.data(), sizeof(float) * nc, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        return hip_fail(e);
    }
    g_offset.emplace(key, d);
    *out = d;
    return XCT_OK;
}

// Checks shared by the offset-scan entry points.
int check_offset(const xct_geometry *g, double overlap)
{
    const double m = 2.0 * g->center;
    if (std::fabs(m - std::nearbyint(m)) > 1e-9) return XCT_EINVAL;
    if (g->center < 0.0 || g->center > g->n_det - 1) return XCT_EINVAL;
    const double short_side = std::min(g->center, (g->n_det - 1) - g->center);
    if (!std::isfinite(overlap) || !(overlap > 0.0) || overlap > short_side + 1e-9) return XCT_EINVAL;
    return XCT_OK;
}

// Forward-projector plan of a geometry (angle table, angle blocks, staging
// shape), built on the host in FP64 and cached on the device.
int fp_tables(const xct_geometry *g, FPTables *out)
{
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::string key;
    key_append(key, dev);
    key_append(key, g->pixel_size / g->det_pitch);
    key_append(key, g->center);
    key_append(key, g->nx);
    key_append(key, g->ny);
    key_append(key, g->n_det);
    key.append(reinterpret_cast<const char *>(g->angles), sizeof(double) * g->n_angles);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_fp.find(key);
    if (it != g_fp.end()) {
        *out = it->second;
        return XCT_OK;
    }
    std::vector<FPAngle> ang;
    std::vector<FPBlock> blocks;
    FPTables t;
    if (int rc = fp_plan(g, ang, blocks, 1, &t.rows[0], &t.pitch[0])) return rc;
    // four slices per workgroup when their staging fits (not for strips many
    // pixels wide)
    if (fp_plan(g, ang, blocks, 4, &t.rows[1], &t.pitch[1]) != XCT_OK) t.rows[1] = 0;
    t.n_blocks = (int)blocks.size();
    hipError_t e = hipMalloc(&t.ang, sizeof(FPAngle) * ang.size());
    if (e == hipSuccess) e = hipMalloc(&t.blocks, sizeof(FPBlock) * blocks.size());
    if (e == hipSuccess)
        e = hipMemcpy(t.ang, ang.data(), sizeof(FPAngle) * ang.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t.blocks, blocks.data(), sizeof(FPBlock) * blocks.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (t.ang) (void)hipFree(t.ang);
        if (t.blocks) (void)hipFree(t.blocks);
        return hip_fail(e);
    }
    g_fp.emplace(key, t);
    *out = t;
    return XCT_OK;
}

// Spatial ramp kernel taps h_W[n] (inverse DTFT of |nu| W(nu) on |nu| <= 1/2).
double ramp_tap(int window, long n)
{
    auto rl = [](long m) -> double {
        if (m == 0) return 0.25;
        if (m % 2 == 0) return 0.0;
        return -1.0 / (M_PI * M_PI * (double)m * (double)m);
    };
    if (window == XCT_RAM_LAK) return rl(n);
    if (window == XCT_SHEPP_LOGAN) return 2.0 / (M_PI * M_PI * (1.0 - 4.0 * (double)n * (double)n));
    return 0.5 * rl(n) + 0.25 * (rl(n - 1) + rl(n + 1));
}

// In-place iterative radix-2 FFT in FP64 (forward, e^{-2 pi i k n / L}).
void host_fft(std::vector<std::complex<double>> &a)
{
    const size_t L = a.size();
    for (size_t i = 1, j = 0; i < L; ++i) {
        size_t bit = L >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= L; len <<= 1) {
        const size_t h = len >> 1;
        for (size_t k = 0; k < h; ++k) {
            const double ang = -2.0 * M_PI * (double)k / (double)len;
            const std::complex<double> w(std::cos(ang), std::sin(ang));
            for (size_t i = 0; i < L; i += len) {
                const std::complex<double> u = a[i + k], v = a[i + k + h] * w;
                a[i + k] = u + v;
                a[i + k + h] = u - v;
            }
        }
    }
}

int fft_length(int nc, int *log2L)
{
    int L = 64, lg = 6;
    while (L < 2 * nc - 1) {
        L <<= 1;
        ++lg;
    }
    *log2L = lg;
    return L;
}

// Twiddles exp(-2 pi i e / L) and the filter spectrum H = DFT_L(h_W placed
// circularly) / (L pitch), both rounded once from FP64.
int filter_tables(int nc, int window, double pitch, FilterTables *out, int *L_out, int *lg_out)
{
    int dev;
    if (int rc = current_device(&dev)) return rc;
    int lg;
    const int L = fft_length(nc, &lg);
    std::string key;
    key_append(key, dev);
    key_append(key, nc);
    key_append(key, window);
    key_append(key, pitch);
    *L_out = L;
    *lg_out = lg;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_filt.find(key);
    if (it != g_filt.end()) {
        *out = it->second;
        return XCT_OK;
    }
    std::vector<std::complex<double>> h(L, 0.0);
    for (long d = -(long)(nc - 1); d <= (long)(nc - 1); ++d)
        h[(size_t)((d % L + L) % L)] = ramp_tap(window, d);
    host_fft(h);
    std::vector<float> H(L);
    for (int k = 0; k < L; ++k) H[k] = (float)(h[k].real() / ((double)L * pitch));
    std::vector<float2> tw(L);
    for (int e = 0; e < L; ++e) {
        const double ang = 2.0 * M_PI * (double)e / (double)L;
        tw[e] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
    }
    FilterTables t;
    hipError_t e = hipMalloc(&t.tw, sizeof(float2) * L);
    if (e == hipSuccess) e = hipMalloc(&t.H, sizeof(float) * L);
    if (e == hipSuccess) e = hipMemcpy(t.tw, tw.data(), sizeof(float2) * L, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(t.H, H.data(), sizeof(float) * L, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (t.tw) (void)hipFree(t.tw);
        if (t.H) (void)hipFree(t.H);
        return hip_fail(e);
    }
    g_filt.emplace(key, t);
    *out = t;
    return XCT_OK;
}

int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

// ---------------------------------------------------------------- back-projection plan

// Window entries per angle for a 64-pixel tile: the detector footprint of the
// tile spans 63 (|C| + |S|) <= 63 sqrt(2) pixel/pitch bins; 3 more cover the
// floor, the right tap and the one-bin margin of the anchor.
int window_entries(double ratio) { return (int)std::ceil((kTile - 1) * std::sqrt(2.0) * ratio + 1e-3) + 3; }

// Half-turn sets of a symmetric angle set: 1 when angle k + N_p/2 is angle k
// plus a quarter turn for every k < N_p/2 (a half turn); 2 when each half of
// the angles is such a set (a full turn, as in offset scans); 0 otherwise,
// or when the slice is not square and even, 2c is not integral, or the
// windows do not fit the symmetric kernel.
int symmetric_sets(const xct_geometry *g)
{
    if (g->nx != g->ny || (g->nx & 1) || (g->n_angles & 1)) return 0;
    if (!bp_sym_window(window_entries(g->pixel_size / g->det_pitch))) return 0;
    const double m = 2.0 * g->center;
    if (std::fabs(m - std::nearbyint(m)) > 1e-9) return 0;
    auto quarter_closed = [g](int k_begin, int n) {
        const int H = n / 2;
        for (int k = 0; k < H; ++k)
            if (std::fabs(g->angles[k_begin + k + H] - g->angles[k_begin + k] - 0.5 * M_PI) > 1e-9)
                return false;
        return true;
    };
    const int np = g->n_angles;
    if (quarter_closed(0, np)) return 1;
    if (np % 4 == 0 && quarter_closed(0, np / 2) && quarter_closed(np / 2, np / 2)) return 2;
    return 0;
}

int choose_path(const xct_geometry *g) { return symmetric_sets(g) ? kPathSymmetric : kPathGeneric; }

struct BPJob {
    const xct_geometry *g;
    GeoTables t;
    int32_t n_slices;
    const void *sino;
    void *image;
    float scale;
    int32_t accumulate;
    int path;
    int32_t out_u16 = 0;
    float code_a = 0.0f, code_b = 0.0f;
};

// Tiles per slice as the kernel indexes them (tiles_x, tiles_y) and the work
// items of the whole slab.
int64_t plan_tiles(const BPJob &j, int sl, int *tx, int *ty)
{
    if (j.path == kPathGeneric) {
        *tx = (j.g->nx + kTile - 1) / kTile;
        *ty = (j.g->ny + kTile - 1) / kTile;
        return (int64_t)*tx * *ty * j.n_slices;
    }
    const int q = (j.g->nx / 2 + kTile - 1) / kTile;  // tiles along a quadrant edge
    *tx = *ty = q;
    return (int64_t)q * q * ((j.n_slices + sl - 1) / sl);
}

// LDS bytes of one angle stage: the symmetric kernel takes 6 angle pairs of
// 8 FP32 windows of 96 entries per slice (four 256-thread or two 512-thread
// workgroups per CU fit in 160 KiB).
#ifndef XCT_SYM2_STAGE_KB
#define XCT_SYM2_STAGE_KB 74
#endif
#ifndef XCT_SYM_MAX_SLICES
#define XCT_SYM_MAX_SLICES 2  // slices per work item of the symmetric kernel (1 or 2)
#endif
constexpr size_t kGenericStageBytes = 32 * 1024;
constexpr size_t kSymStageBytes = 37 * 1024;
constexpr size_t kSym2StageBytes = XCT_SYM2_STAGE_KB * 1024;

// Launch one back-projection over jobs that all take the same kernel path.
// counter != nullptr makes it persistent.
int launch_bp_jobs(std::vector<BPJob> jobs, int dtype, unsigned int *counter, hipStream_t s)
{
    if (jobs.empty()) return XCT_OK;
    const int path = jobs[0].path;
    // largest cost per item first (items of one slab cost the same)
    std::stable_sort(jobs.begin(), jobs.end(),
                     [](const BPJob &a, const BPJob &b) { return a.g->n_angles > b.g->n_angles; });
    // two slices per work item when every slab has at least two
    int spi = path == kPathSymmetric ? XCT_SYM_MAX_SLICES : 1;
    for (const BPJob &j : jobs)
        if (j.n_slices < 2) spi = 1;
    BPBatch b;
    std::memset(&b, 0, sizeof(b));
    int W = 0;
    int64_t items = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        const BPJob &j = jobs[i];
        BPSlab &sl = b.slab[i];
        int tx, ty;
        const int64_t n_items = plan_tiles(j, spi, &tx, &ty);
        sl.sino = j.sino;
        sl.image = j.image;
        sl.cs = j.t.cs;
        sl.csd = j.t.csd;
        sl.center = j.g->center;
        sl.item_begin = items;
        sl.n_angles = j.g->n_angles;
        sl.n_det = j.g->n_det;
        sl.nx = j.g->nx;
        sl.ny = j.g->ny;
        sl.n_slices = j.n_slices;
        sl.tiles_x = tx;
        sl.tiles_y = ty;
        sl.mirror = path != kPathGeneric ? (int32_t)std::nearbyint(2.0 * j.g->center) : 0;
        sl.sets = path != kPathGeneric ? symmetric_sets(j.g) : 1;
        sl.scale = j.scale;
        sl.accumulate = j.accumulate;
        sl.out_u16 = j.out_u16;
        sl.code_a = j.code_a;
        sl.code_b = j.code_b;
        items += n_items;
        W = std::max(W, window_entries(j.g->pixel_size / j.g->det_pitch));
    }
    if (items >= (int64_t)1 << 31) return XCT_ETOOBIG;
    b.n_slabs = (int32_t)jobs.size();
    b.total_items = items;
    b.counter = counter;
    size_t lds;
    if (path == kPathSymmetric) {
        W = bp_sym_window(W);  // choose_path only routes windows that fit here
        const size_t budget = spi == 2 ? kSym2StageBytes : kSymStageBytes;
        b.kb = (int)std::max<size_t>(1, budget / (4 * (size_t)W * spi * sizeof(float4) + 24));
        lds = bp_sym_lds_bytes(W, b.kb, spi);
    } else {
        b.kb = (int)std::max<size_t>(1, std::min<size_t>(64, kGenericStageBytes / (8 * (size_t)W + 16)));
        lds = bp_generic_lds_bytes(W, b.kb);
    }
    b.win = W;
    if (lds > 160 * 1024) return XCT_ETOOBIG;
    int grid;
    if (counter) {
        const int per_cu = bp_max_blocks_per_cu(path, dtype, W, spi, lds);
        grid = (int)std::min<int64_t>(items, (int64_t)per_cu * device_cus());
        b.xcd_remap = 0;
    } else {
        grid = (int)items;
        b.xcd_remap = (items % 8 == 0) ? 1 : 0;
    }
    hipError_t e = launch_bp(path, b, dtype, spi, grid, lds, s);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ================================================================ C ABI

extern "C" {

const char *xct_status_string(int status)
{
    switch (status) {
    case XCT_OK: return "ok";
    case XCT_EINVAL: return "invalid argument";
    case XCT_EDTYPE: return "unsupported dtype or window";
    case XCT_EWORKSPACE: return "workspace missing, misaligned or too small";
    case XCT_ETOOBIG: return "size beyond the supported limits";
    case XCT_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

int xct_version(void) { return XCT_VERSION; }

int xct_last_hip_error(void) { return g_last_hip; }

void xct_cache_clear(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &kv : g_geo) {
        (void)hipFree(kv.second.cs);
        (void)hipFree(kv.second.csd);
    }
    for (auto &kv : g_filt) {
        (void)hipFree(kv.second.tw);
        (void)hipFree(kv.second.H);
    }
    for (auto &kv : g_fp) {
        (void)hipFree(kv.second.ang);
        (void)hipFree(kv.second.blocks);
    }
    for (auto &kv : g_blur) (void)hipFree(kv.second);
    for (auto &kv : g_offset) (void)hipFree(kv.second);
    g_offset.clear();
    g_geo.clear();
    g_filt.clear();
    g_fp.clear();
    g_blur.clear();
}

int xct_filter(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
               void *filtered, int32_t filtered_t, int32_t window, xct_stream stream)
{
    if (int rc = check_geometry(g, false)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (!sino || !filtered) return XCT_EINVAL;
    if (!dtype_ok(sino_t) || !dtype_ok(filtered_t)) return XCT_EDTYPE;
    if (window < XCT_RAM_LAK || window > XCT_HANN) return XCT_EDTYPE;
    if (sino == filtered && sino_t != filtered_t) return XCT_EINVAL;
    if (g->n_det > kMaxFFT / 2) return XCT_ETOOBIG;
    FilterTables ft;
    int L, lg;
    if (int rc = filter_tables(g->n_det, window, g->det_pitch, &ft, &L, &lg)) return rc;
    FilterArgs a{};
    a.in = sino;
    a.out = filtered;
    a.tw = ft.tw;
    a.H = ft.H;
    a.rows = (int64_t)n_slices * g->n_angles;
    a.nc = g->n_det;
    a.in_len = g->n_det;
    a.L = L;
    a.log2L = lg;
    hipError_t e = launch_filter(a, sino_t, filtered_t, (hipStream_t)stream);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

int xct_offset_detector(const xct_geometry *g, int32_t *n_virtual, double *center_virtual)
{
    if (int rc = check_geometry(g, false)) return rc;
    if (!n_virtual || !center_virtual) return XCT_EINVAL;
    const double m = 2.0 * g->center;
    if (std::fabs(m - std::nearbyint(m)) > 1e-9) return XCT_EINVAL;
    if (g->center < 0.0 || g->center > g->n_det - 1) return XCT_EINVAL;
    int nv, first;
    double cv;
    offset_virtual(g, &nv, &cv, &first);
    *n_virtual = nv;
    *center_virtual = cv;
    return XCT_OK;
}

int xct_filter_offset(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
                      void *filtered, int32_t filtered_t, int32_t window, double overlap,
                      xct_stream stream)
{
    if (int rc = check_geometry(g, false)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (!sino || !filtered || sino == filtered) return XCT_EINVAL;
    if (!dtype_ok(sino_t) || !dtype_ok(filtered_t)) return XCT_EDTYPE;
    if (window < XCT_RAM_LAK || window > XCT_HANN) return XCT_EDTYPE;
    if (int rc = check_offset(g, overlap)) return rc;
    int nv, first;
    double cv;
    offset_virtual(g, &nv, &cv, &first);
    if (nv > kMaxFFT / 2) return XCT_ETOOBIG;
    FilterTables ft;
    int L, lg;
    if (int rc = filter_tables(nv, window, g->det_pitch, &ft, &L, &lg)) return rc;
    const float *w = nullptr;
    if (int rc = offset_weights(g, overlap, &w)) return rc;
    FilterArgs a{};
    a.in = sino;
    a.out = filtered;
    a.tw = ft.tw;
    a.H = ft.H;
    a.weight = w;
    a.in_first = first;
    a.in_len = g->n_det;
    a.rows = (int64_t)n_slices * g->n_angles;
    a.nc = nv;
    a.L = L;
    a.log2L = lg;
    hipError_t e = launch_filter(a, sino_t, filtered_t, (hipStream_t)stream);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

int xct_preprocess_filter(const xct_geometry *g, int32_t n_rows, int32_t row_begin, int32_t n_slices,
                          const void *proj, int32_t proj_t, const float *dark, const float *flat,
                          float floor, float blur_sigma, void *filtered, int32_t filtered_t,
                          int32_t window, xct_stream stream)
{
    if (int rc = check_geometry(g, false)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (n_rows < 1 || row_begin < 0 || (int64_t)row_begin + n_slices > n_rows) return XCT_EINVAL;
    if (!proj || !dark || !flat || !filtered) return XCT_EINVAL;
    if ((proj_t != XCT_U16 && proj_t != XCT_F32) || !dtype_ok(filtered_t)) return XCT_EDTYPE;
    if (window < XCT_RAM_LAK || window > XCT_HANN) return XCT_EDTYPE;
    if (!std::isfinite(floor) || !(floor > 0.0f)) return XCT_EINVAL;
    if (!std::isfinite(blur_sigma) || blur_sigma < 0.0f) return XCT_EINVAL;
    if (g->n_det > kMaxFFT / 2) return XCT_ETOOBIG;
    const int radius = blur_sigma == 0.0f ? 0 : (int)(4.0 * (double)blur_sigma + 0.5);
    if (radius > 64) return XCT_ETOOBIG;
    // the output must not overlap the projection stack
    const char *pb = static_cast<const char *>(proj), *fb = static_cast<const char *>(filtered);
    const size_t pbytes = (size_t)g->n_angles * n_rows * g->n_det * dtype_size(proj_t);
    const size_t fbytes = (size_t)n_slices * g->n_angles * g->n_det * dtype_size(filtered_t);
    if (pb < fb + fbytes && fb < pb + pbytes) return XCT_EINVAL;
    FilterTables ft;
    int L, lg;
    if (int rc = filter_tables(g->n_det, window, g->det_pitch, &ft, &L, &lg)) return rc;
    const float *taps = nullptr;
    if (radius > 0)
        if (int rc = blur_taps(blur_sigma, radius, &taps)) return rc;
    FilterArgs a{};
    a.in = proj;
    a.out = filtered;
    a.tw = ft.tw;
    a.H = ft.H;
    a.rows = (int64_t)n_slices * g->n_angles;
    a.nc = g->n_det;
    a.L = L;
    a.log2L = lg;
    a.pre.dark = dark;
    a.pre.flat = flat;
    a.pre.taps = taps;
    a.pre.radius = radius;
    a.pre.n_rows = n_rows;
    a.pre.row_begin = row_begin;
    a.pre.n_angles = g->n_angles;
    a.pre.floor = floor;
    hipError_t e = launch_front_end_filter(a, proj_t, filtered_t, (hipStream_t)stream);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

int xct_backproject(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
                    float *image, float scale, int32_t accumulate, xct_stream stream)
{
    if (int rc = check_geometry(g, true)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (!sino || !image) return XCT_EINVAL;
    if (!dtype_ok(sino_t)) return XCT_EDTYPE;
    if (!std::isfinite(scale)) return XCT_EINVAL;
    BPJob j;
    j.g = g;
    j.n_slices = n_slices;
    j.sino = sino;
    j.image = image;
    j.scale = scale;
    j.accumulate = accumulate ? 1 : 0;
    j.path = choose_path(g);
    if (int rc = geo_tables(g, &j.t)) return rc;
    return launch_bp_jobs({j}, sino_t, nullptr, (hipStream_t)stream);
}

int xct_backproject_u16(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
                        uint16_t *image, float scale, double mu_water, double hu_min, double hu_max,
                        xct_stream stream)
{
    if (int rc = check_geometry(g, true)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (!sino || !image) return XCT_EINVAL;
    if (!dtype_ok(sino_t)) return XCT_EDTYPE;
    if (!std::isfinite(scale) || !std::isfinite(mu_water) || !std::isfinite(hu_min) ||
        !std::isfinite(hu_max) || !(mu_water > 0.0) || !(hu_max > hu_min))
        return XCT_EINVAL;
    // code = A mu + B: HU = 1000 (mu - mu_water) / mu_water, [hu_min, hu_max] -> [0, 65535]
    const double span = 65535.0 / (hu_max - hu_min);
    const double A = 1000.0 / mu_water * span;
    const double B = (-1000.0 - hu_min) * span;
    const float a32 = (float)A, b32 = (float)B;
    if (!std::isfinite(a32) || !std::isfinite(b32)) return XCT_EINVAL;
    BPJob j;
    j.g = g;
    j.n_slices = n_slices;
    j.sino = sino;
    j.image = image;
    j.scale = scale;
    j.accumulate = 0;
    j.path = choose_path(g);
    j.out_u16 = 1;
    j.code_a = a32;
    j.code_b = b32;
    if (int rc = geo_tables(g, &j.t)) return rc;
    return launch_bp_jobs({j}, sino_t, nullptr, (hipStream_t)stream);
}

int xct_forward_project(const xct_geometry *g, int32_t n_slices, const float *image, float *sino,
                        float scale, int32_t accumulate, xct_stream stream)
{
    if (int rc = check_geometry(g, true)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (!image || !sino) return XCT_EINVAL;
    if (!std::isfinite(scale)) return XCT_EINVAL;
    if (n_slices > 65535) return XCT_ETOOBIG;
    FPTables t;
    if (int rc = fp_tables(g, &t)) return rc;
    FPArgs a;
    a.image = image;
    a.sino = sino;
    a.ang = t.ang;
    a.blocks = t.blocks;
    a.n_blocks = t.n_blocks;
    a.bin_blocks = (g->n_det + kFPBins - 1) / kFPBins;
    // four slices per workgroup share coordinates and weights; a call with
    // one or two slices keeps one per workgroup
    const int sl = (n_slices >= 3 && t.rows[1] > 0) ? 4 : 1;
    a.rows = t.rows[sl == 4];
    a.pitch = t.pitch[sl == 4];
    a.scale = scale;
    a.accumulate = accumulate ? 1 : 0;
    a.n_angles = g->n_angles;
    a.n_det = g->n_det;
    a.nx = g->nx;
    a.ny = g->ny;
    a.n_slices = n_slices;
    hipError_t e = launch_forward(a, sl, (hipStream_t)stream);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

// Detector bins of a slab's filtered rows: the virtual (mirrored) detector
// for an offset scan, the physical one otherwise.
static int filtered_bins(const xct_slab &sl)
{
    if (sl.offset_overlap == 0.0) return sl.geom.n_det;
    int nv, first;
    double cv;
    offset_virtual(&sl.geom, &nv, &cv, &first);
    return nv;
}

static int check_slabs(const xct_slab *slabs, int32_t n_slabs, bool need_data)
{
    if (!slabs || n_slabs <= 0) return XCT_EINVAL;
    if (n_slabs > kMaxSlabs) return XCT_ETOOBIG;
    for (int i = 0; i < n_slabs; ++i) {
        if (int rc = check_geometry(&slabs[i].geom, true)) return rc;
        if (int rc = check_slices(&slabs[i].geom, slabs[i].n_slices)) return rc;
        if (slabs[i].offset_overlap != 0.0)
            if (int rc = check_offset(&slabs[i].geom, slabs[i].offset_overlap)) return rc;
        if (filtered_bins(slabs[i]) > kMaxFFT / 2) return XCT_ETOOBIG;
        if (need_data && (!slabs[i].sino || !slabs[i].image)) return XCT_EINVAL;
    }
    return XCT_OK;
}

size_t xct_fbp_workspace_bytes(const xct_slab *slabs, int32_t n_slabs, int32_t filtered_t)
{
    if (check_slabs(slabs, n_slabs, false) || !dtype_ok(filtered_t)) return 0;
    size_t bytes = 256;  // work counters
    for (int i = 0; i < n_slabs; ++i) {
        const xct_geometry &g = slabs[i].geom;
        bytes += align256((size_t)slabs[i].n_slices * g.n_angles * filtered_bins(slabs[i]) *
                          dtype_size(filtered_t));
    }
    return bytes;
}

int xct_fbp_batch(const xct_slab *slabs, int32_t n_slabs, int32_t sino_t, int32_t window,
                  int32_t filtered_t, void *workspace, size_t workspace_bytes, xct_stream stream)
{
    if (int rc = check_slabs(slabs, n_slabs, true)) return rc;
    if (!dtype_ok(sino_t) || !dtype_ok(filtered_t)) return XCT_EDTYPE;
    if (window < XCT_RAM_LAK || window > XCT_HANN) return XCT_EDTYPE;
    const size_t need = xct_fbp_workspace_bytes(slabs, n_slabs, filtered_t);
    if (!workspace || ((uintptr_t)workspace & 255) || workspace_bytes < need) return XCT_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;

    char *ws = static_cast<char *>(workspace);
    unsigned int *counters = reinterpret_cast<unsigned int *>(ws);
    size_t off = 256;
    std::vector<BPJob> jobs_by_path[2];
    // back-projection geometry of offset slabs (virtual detector); lives until
    // the launches below have read it
    std::vector<xct_geometry> virt(n_slabs);
    for (int i = 0; i < n_slabs; ++i) {
        const xct_slab &sl = slabs[i];
        const xct_geometry *g = &sl.geom;
        void *filt = ws + off;
        off += align256((size_t)sl.n_slices * g->n_angles * filtered_bins(sl) * dtype_size(filtered_t));
        double weight = M_PI / g->n_angles;
        if (sl.offset_overlap != 0.0) {
            // full-turn offset scan: redundancy-weighted rows filtered on the
            // virtual detector, back-projected with weight 2 pi / N_p
            if (int rc = xct_filter_offset(g, sl.n_slices, sl.sino, sino_t, filt, filtered_t, window,
                                           sl.offset_overlap, stream))
                return rc;
            int first;
            virt[i] = *g;
            offset_virtual(g, &virt[i].n_det, &virt[i].center, &first);
            g = &virt[i];
            weight = 2.0 * M_PI / g->n_angles;
        } else if (int rc = xct_filter(g, sl.n_slices, sl.sino, sino_t, filt, filtered_t, window, stream)) {
            return rc;
        }
        BPJob j;
        j.g = g;
        j.n_slices = sl.n_slices;
        j.sino = filt;
        j.image = sl.image;
        j.scale = (float)weight;
        j.accumulate = 0;
        j.path = choose_path(g);
        if (int rc = geo_tables(g, &j.t)) return rc;
        jobs_by_path[j.path].push_back(j);
    }
    hipError_t e = launch_fill_u32(counters, 2, 0u, s);
    if (e != hipSuccess) return hip_fail(e);
    for (int p = kPathSymmetric; p >= kPathGeneric; --p)
        if (int rc = launch_bp_jobs(jobs_by_path[p], filtered_t, counters + p, s)) return rc;
    return XCT_OK;
}

size_t xct_reduce_workspace_bytes(int64_t n)
{
    if (n <= 0) return 0;
    return sizeof(double) * (size_t)reduce_blocks(n);
}

static int reduce_common(const float *a, const float *b, int64_t n, double *result, void *workspace,
                         size_t workspace_bytes, int sqdist, xct_stream stream)
{
    if (!a || !b || !result || n <= 0) return XCT_EINVAL;
    if (!workspace || ((uintptr_t)workspace & 7) || workspace_bytes < xct_reduce_workspace_bytes(n))
        return XCT_EWORKSPACE;
    hipError_t e = launch_reduce(a, b, n, result, static_cast<double *>(workspace), reduce_blocks(n),
                                 sqdist, (hipStream_t)stream);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

int xct_dot_f64(const float *a, const float *b, int64_t n, double *result, void *workspace,
                size_t workspace_bytes, xct_stream stream)
{
    return reduce_common(a, b, n, result, workspace, workspace_bytes, 0, stream);
}

int xct_sqdist_f64(const float *a, const float *b, int64_t n, double *result, void *workspace,
                   size_t workspace_bytes, xct_stream stream)
{
    return reduce_common(a, b, n, result, workspace, workspace_bytes, 1, stream);
}

}  // extern "C"
