// C ABI of libxct.so: argument validation, per-geometry device tables and
// dispatch of the filter, back-projection, forward-projection and reduction
// kernels.  See include/xct.h for the contract of every entry point.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <memory>
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

// Stream-ordered scratch of the forward projector's four-slice copies: at
// most this much per chunk, and the device's default pool keeps up to this
// much between calls instead of returning it at each synchronisation.
constexpr int64_t kQuadBytes = (int64_t)1 << 30;

void keep_stream_pool()
{
    static std::mutex m;
    static std::vector<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(m);
    if (std::find(done.begin(), done.end(), dev) != done.end()) return;
    done.push_back(dev);
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
    uint64_t keep = (uint64_t)kQuadBytes;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
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
//
// Per-geometry tables (trigonometry, filter spectra, forward-projector plans,
// blur taps, redundancy weights) are built on the host in FP64 and cached on
// the device.  One cache entry is one device allocation holding its tables at
// 256-byte offsets.  Its upload is ordered on the stream of the call that
// creates it (an asynchronous copy from pinned host staging, kept with the
// entry), and an event marks its completion so that calls on other streams
// wait for it.  The cache is bounded: past kCacheEntries entries or
// kCacheBytes bytes the least recently used entries that no call is using are
// freed (hipFree, which waits for the device).

constexpr size_t kCacheBytes = (size_t)1 << 30;
constexpr size_t kCacheEntries = 256;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Entry {
    char *dev = nullptr;        // device allocation (all tables of the entry)
    void *host = nullptr;       // pinned staging of the upload
    hipEvent_t ready = nullptr; // recorded after the upload, on the creating call's stream
    bool done = false;          // the upload is known to be complete
    size_t bytes = 0;
    uint64_t tick = 0;
    size_t off[2] = {0, 0};     // offsets of the entry's tables in `dev`
    // forward-projector plan metadata
    int n_blocks = 0;
    bool fp_four = false;  // every angle block has a four-slice staging shape
    // filter length
    int L = 0, lg = 0;
    template <typename T>
    T *table(int i) const { return reinterpret_cast<T *>(dev + off[i]); }
};
typedef std::shared_ptr<Entry> EntryRef;

std::mutex g_mu;
std::unordered_map<std::string, EntryRef> g_cache;
size_t g_cache_bytes = 0;
uint64_t g_tick = 0;

void entry_release(Entry &e)
{
    if (e.dev) (void)hipFree(e.dev);
    if (e.host) (void)hipHostFree(e.host);
    if (e.ready) (void)hipEventDestroy(e.ready);
    e.dev = nullptr;
    e.host = nullptr;
    e.ready = nullptr;
}

// Evict least recently used entries held by no call until `incoming` more
// bytes fit (called with g_mu held).
void cache_make_room(size_t incoming)
{
    while (!g_cache.empty() &&
           (g_cache.size() + 1 > kCacheEntries || g_cache_bytes + incoming > kCacheBytes)) {
        auto victim = g_cache.end();
        for (auto it = g_cache.begin(); it != g_cache.end(); ++it)
            if (it->second.use_count() == 1 && (victim == g_cache.end() || it->second->tick < victim->second->tick))
                victim = it;
        if (victim == g_cache.end()) return;  // every entry is in use: grow past the bound
        (void)hipDeviceSynchronize();         // kernels of earlier calls may still read it
        g_cache_bytes -= victim->second->bytes;
        entry_release(*victim->second);
        g_cache.erase(victim);
    }
}

// Look up `key`; on a hit whose upload may still be in flight, make
// `stream` wait for it.  *out is empty on a miss.  Called with g_mu held.
int cache_find(const std::string &key, hipStream_t stream, EntryRef *out)
{
    auto it = g_cache.find(key);
    if (it == g_cache.end()) {
        out->reset();
        return XCT_OK;
    }
    Entry &e = *it->second;
    e.tick = ++g_tick;
    if (!e.done) {
        hipError_t q = hipEventQuery(e.ready);
        if (q == hipSuccess) {
            e.done = true;
        } else if (q == hipErrorNotReady) {
            hipError_t w = hipStreamWaitEvent(stream, e.ready, 0);
            if (w != hipSuccess) return hip_fail(w);
        } else {
            return hip_fail(q);
        }
    }
    *out = it->second;
    return XCT_OK;
}

// Create and upload an entry from host tables `parts` (up to two), ordered on
// `stream`.  Called with g_mu held.
int cache_insert(const std::string &key, const void *const parts[2], const size_t sizes[2],
                 hipStream_t stream, const Entry &meta, EntryRef *out)
{
    EntryRef e = std::make_shared<Entry>(meta);
    size_t total = 0;
    for (int i = 0; i < 2; ++i) {
        e->off[i] = total;
        total += align256(sizes[i]);
    }
    total = std::max<size_t>(total, 256);
    cache_make_room(total);
    hipError_t r = hipMalloc(reinterpret_cast<void **>(&e->dev), total);
    if (r == hipSuccess) r = hipHostMalloc(&e->host, total, hipHostMallocDefault);
    if (r == hipSuccess) {
        for (int i = 0; i < 2; ++i)
            if (sizes[i]) std::memcpy(static_cast<char *>(e->host) + e->off[i], parts[i], sizes[i]);
        r = hipMemcpyAsync(e->dev, e->host, total, hipMemcpyHostToDevice, stream);
    }
    if (r == hipSuccess) r = hipEventCreateWithFlags(&e->ready, hipEventDisableTiming);
    if (r == hipSuccess) r = hipEventRecord(e->ready, stream);
    if (r != hipSuccess) {
        entry_release(*e);
        return hip_fail(r);
    }
    e->bytes = total;
    e->tick = ++g_tick;
    g_cache.emplace(key, e);
    g_cache_bytes += total;
    *out = e;
    return XCT_OK;
}

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

// Key prefix: kind, device.
int cache_key(char kind, std::string &key)
{
    int dev;
    if (int rc = current_device(&dev)) return rc;
    key.clear();
    key.push_back(kind);
    key_append(key, dev);
    return XCT_OK;
}

// cos/sin of every angle times pixel/pitch, in FP32 (inner loops, table 0) and
// FP64 (window anchors, table 1), rounded once from FP64 host trigonometry.
int geo_tables(const xct_geometry *g, hipStream_t stream, EntryRef *out)
{
    std::string key;
    if (int rc = cache_key('g', key)) return rc;
    const double r = g->pixel_size / g->det_pitch;
    key_append(key, r);
    key.append(reinterpret_cast<const char *>(g->angles), sizeof(double) * g->n_angles);
    std::lock_guard<std::mutex> lock(g_mu);
    if (int rc = cache_find(key, stream, out)) return rc;
    if (*out) return XCT_OK;
    const int n = g->n_angles;
    std::vector<float2> cs(n);
    std::vector<double2> csd(n);
    for (int k = 0; k < n; ++k) {
        const double c = std::cos(g->angles[k]) * r, s = std::sin(g->angles[k]) * r;
        csd[k] = make_double2(c, s);
        cs[k] = make_float2((float)c, (float)s);
    }
    const void *parts[2] = {cs.data(), csd.data()};
    const size_t sizes[2] = {sizeof(float2) * n, sizeof(double2) * n};
    return cache_insert(key, parts, sizes, stream, Entry(), out);
}

// Unit-sum sampled Gaussian of standard deviation sigma over -R..R,
// R = int(4 sigma + 0.5), in FP64 rounded once to FP32.
int blur_taps(float sigma, int radius, hipStream_t stream, EntryRef *out)
{
    std::string key;
    if (int rc = cache_key('b', key)) return rc;
    key_append(key, sigma);
    std::lock_guard<std::mutex> lock(g_mu);
    if (int rc = cache_find(key, stream, out)) return rc;
    if (*out) return XCT_OK;
    std::vector<double> g(2 * radius + 1);
    double sum = 0.0;
    for (int m = -radius; m <= radius; ++m) {
        const double t = (double)m / (double)sigma;
        g[m + radius] = std::exp(-0.5 * t * t);
        sum += g[m + radius];
    }
    std::vector<float> g32(g.size());
    for (size_t i = 0; i < g.size(); ++i) g32[i] = (float)(g[i] / sum);
    const void *parts[2] = {g32.data(), nullptr};
    const size_t sizes[2] = {sizeof(float) * g32.size(), 0};
    return cache_insert(key, parts, sizes, stream, Entry(), out);
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
// one together.  FP64 on the host, rounded once.
int offset_weights(const xct_geometry *g, double overlap, hipStream_t stream, EntryRef *out)
{
    std::string key;
    if (int rc = cache_key('o', key)) return rc;
    key_append(key, g->n_det);
    key_append(key, g->center);
    key_append(key, overlap);
    std::lock_guard<std::mutex> lock(g_mu);
    if (int rc = cache_find(key, stream, out)) return rc;
    if (*out) return XCT_OK;
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
    const void *parts[2] = {w.data(), nullptr};
    const size_t sizes[2] = {sizeof(float) * nc, 0};
    return cache_insert(key, parts, sizes, stream, Entry(), out);
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

// Forward-projector plan of a geometry (angle table 0, angle blocks 1, the
// staging shapes for one and four slices per workgroup).
int fp_tables(const xct_geometry *g, hipStream_t stream, EntryRef *out)
{
    std::string key;
    if (int rc = cache_key('f', key)) return rc;
    key_append(key, g->pixel_size / g->det_pitch);
    key_append(key, g->center);
    key_append(key, g->nx);
    key_append(key, g->ny);
    key_append(key, g->n_det);
    key.append(reinterpret_cast<const char *>(g->angles), sizeof(double) * g->n_angles);
    std::lock_guard<std::mutex> lock(g_mu);
    if (int rc = cache_find(key, stream, out)) return rc;
    if (*out) return XCT_OK;
    std::vector<FPAngle> ang;
    std::vector<FPBlock> blocks;
    Entry meta;
    // four slices per workgroup when their staging fits (not for strips many
    // pixels wide)
    if (int rc = fp_plan(g, ang, blocks, &meta.fp_four)) return rc;
    meta.n_blocks = (int)blocks.size();
    const void *parts[2] = {ang.data(), blocks.data()};
    const size_t sizes[2] = {sizeof(FPAngle) * ang.size(), sizeof(FPBlock) * blocks.size()};
    return cache_insert(key, parts, sizes, stream, meta, out);
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

// Twiddles exp(-2 pi i e / L) (table 0) and the filter spectrum H =
// DFT_L(h_W placed circularly) / (L pitch) (table 1), both rounded once from
// FP64.
int filter_tables(int nc, int window, double pitch, hipStream_t stream, EntryRef *out)
{
    std::string key;
    if (int rc = cache_key('h', key)) return rc;
    key_append(key, nc);
    key_append(key, window);
    key_append(key, pitch);
    std::lock_guard<std::mutex> lock(g_mu);
    if (int rc = cache_find(key, stream, out)) return rc;
    if (*out) return XCT_OK;
    Entry meta;
    const int L = fft_length(nc, &meta.lg);
    meta.L = L;
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
    const void *parts[2] = {tw.data(), H.data()};
    const size_t sizes[2] = {sizeof(float2) * L, sizeof(float) * L};
    return cache_insert(key, parts, sizes, stream, meta, out);
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

// Kernel path of a geometry: the quarter-turn + mirror symmetric kernel when
// it applies; otherwise the mirror kernel when 2c is integral (detector bin
// 2c - n exists for every bin n) and its windows fit; otherwise the generic
// kernel.
int choose_path(const xct_geometry *g)
{
    if (symmetric_sets(g)) return kPathSymmetric;
    const double m = 2.0 * g->center;
    if (std::fabs(m - std::nearbyint(m)) <= 1e-9 && bp_sym_window(window_entries(g->pixel_size / g->det_pitch)))
        return kPathMirror;
    return kPathGeneric;
}

struct BPJob {
    const xct_geometry *g;  // geometry the rows are back-projected with
    EntryRef t;             // its trigonometry tables
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
    if (j.path == kPathMirror) {  // the upper ceil(N_y/2) rows
        *tx = (j.g->nx + kTile - 1) / kTile;
        *ty = ((j.g->ny + 1) / 2 + kTile - 1) / kTile;
        return (int64_t)*tx * *ty * ((j.n_slices + sl - 1) / sl);
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
// `counters` (kXcds zeroed words on the stream) makes it persistent; `table`
// is device memory for the slab descriptors, needed when there are more than
// kInlineSlabs jobs.  A non-persistent launch whose grid would exceed 2^32
// work-items is split into several launches over consecutive item ranges.
int launch_bp_jobs(std::vector<BPJob> jobs, int dtype, unsigned int *counters, BPSlab *table,
                   hipStream_t s)
{
    if (jobs.empty()) return XCT_OK;
    const int path = jobs[0].path;
    // largest cost per item first (items of one slab cost the same)
    std::stable_sort(jobs.begin(), jobs.end(),
                     [](const BPJob &a, const BPJob &b) { return a.g->n_angles > b.g->n_angles; });
    // two slices per work item when every slab has at least two
    int spi = path != kPathGeneric ? XCT_SYM_MAX_SLICES : 1;
    for (const BPJob &j : jobs)
        if (j.n_slices < 2) spi = 1;
    std::vector<BPSlab> desc(jobs.size());
    int W = 0;
    int64_t items = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        const BPJob &j = jobs[i];
        BPSlab &sl = desc[i];
        std::memset(&sl, 0, sizeof(sl));
        int tx, ty;
        const int64_t n_items = plan_tiles(j, spi, &tx, &ty);
        sl.sino = j.sino;
        sl.image = j.image;
        sl.cs = j.t->table<float2>(0);
        sl.csd = j.t->table<double2>(1);
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
        sl.sets = path == kPathSymmetric ? symmetric_sets(j.g) : 1;
        sl.scale = j.scale;
        sl.accumulate = j.accumulate;
        sl.out_u16 = j.out_u16;
        sl.code_a = j.code_a;
        sl.code_b = j.code_b;
        items += n_items;
        W = std::max(W, window_entries(j.g->pixel_size / j.g->det_pitch));
    }
    if (items >= (int64_t)1 << 31) return XCT_ETOOBIG;
    BPBatch b;
    std::memset(&b, 0, sizeof(b));
    b.n_slabs = (int32_t)jobs.size();
    b.total_items = items;
    b.counter = counters;
    size_t lds;
    if (path == kPathSymmetric) {
        W = bp_sym_window(W);  // choose_path only routes windows that fit here
        const size_t budget = spi == 2 ? kSym2StageBytes : kSymStageBytes;
        b.kb = (int)std::max<size_t>(1, budget / (4 * (size_t)W * spi * sizeof(float4) + 24));
        lds = bp_sym_lds_bytes(W, b.kb, spi);
    } else if (path == kPathMirror) {
        W = bp_sym_window(W);
        const size_t budget = spi == 2 ? kSym2StageBytes : kSymStageBytes;
        b.kb = (int)std::max<size_t>(1, budget / ((size_t)W * spi * sizeof(float4) + sizeof(float4)));
        lds = bp_mirror_lds_bytes(W, b.kb, spi);
    } else {
        b.kb = (int)std::max<size_t>(1, std::min<size_t>(64, kGenericStageBytes / (8 * (size_t)W + 16)));
        lds = bp_generic_lds_bytes(W, b.kb);
    }
    b.win = W;
    if (lds > 160 * 1024) return XCT_ETOOBIG;
    if (jobs.size() > (size_t)kInlineSlabs) {
        if (!table) return XCT_ETOOBIG;
        hipError_t e = write_slab_table(table, desc.data(), (int)desc.size(), s);
        if (e != hipSuccess) return hip_fail(e);
        b.table = table;
    } else {
        std::memcpy(b.slab, desc.data(), sizeof(BPSlab) * desc.size());
    }
    if (counters) {
        const int per_cu = bp_max_blocks_per_cu(path, dtype, W, spi, lds);
        const int grid = (int)std::min<int64_t>(items, (int64_t)per_cu * device_cus());
        hipError_t e = launch_bp(path, b, dtype, spi, grid, lds, s);
        return e == hipSuccess ? XCT_OK : hip_fail(e);
    }
    const int64_t threads = bp_block_threads(path, spi);
    const int64_t max_items = ((((int64_t)1 << 32) - 1) / threads) & ~(int64_t)7;
    for (int64_t base = 0; base < items; base += max_items) {
        const int64_t count = std::min(max_items, items - base);
        b.item_base = base;
        b.xcd_remap = (count % 8 == 0) ? 1 : 0;
        hipError_t e = launch_bp(path, b, dtype, spi, (int)count, lds, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    return XCT_OK;
}

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
    for (auto &kv : g_cache) entry_release(*kv.second);
    g_cache.clear();
    g_cache_bytes = 0;
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
    hipStream_t s = (hipStream_t)stream;
    EntryRef ft;
    if (int rc = filter_tables(g->n_det, window, g->det_pitch, s, &ft)) return rc;
    FilterArgs a{};
    a.in = sino;
    a.out = filtered;
    a.tw = ft->table<float2>(0);
    a.H = ft->table<float>(1);
    a.rows = (int64_t)n_slices * g->n_angles;
    a.nc = g->n_det;
    a.in_len = g->n_det;
    a.L = ft->L;
    a.log2L = ft->lg;
    hipError_t e = launch_filter(a, sino_t, filtered_t, s);
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
    hipStream_t s = (hipStream_t)stream;
    EntryRef ft, w;
    if (int rc = filter_tables(nv, window, g->det_pitch, s, &ft)) return rc;
    if (int rc = offset_weights(g, overlap, s, &w)) return rc;
    FilterArgs a{};
    a.in = sino;
    a.out = filtered;
    a.tw = ft->table<float2>(0);
    a.H = ft->table<float>(1);
    a.weight = w->table<float>(0);
    a.in_first = first;
    a.in_len = g->n_det;
    a.rows = (int64_t)n_slices * g->n_angles;
    a.nc = nv;
    a.L = ft->L;
    a.log2L = ft->lg;
    hipError_t e = launch_filter(a, sino_t, filtered_t, s);
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
    if (!std::isfinite(floor) || !(floor >= std::numeric_limits<float>::min())) return XCT_EINVAL;
    if (!std::isfinite(blur_sigma) || blur_sigma < 0.0f) return XCT_EINVAL;
    if (g->n_det > kMaxFFT / 2) return XCT_ETOOBIG;
    if ((double)g->n_angles * n_rows * g->n_det > 4.0e18) return XCT_ETOOBIG;
    const int radius = blur_sigma == 0.0f ? 0 : (int)(4.0 * (double)blur_sigma + 0.5);
    if (radius > 64) return XCT_ETOOBIG;
    // the output must not overlap the projection stack
    const char *pb = static_cast<const char *>(proj), *fb = static_cast<const char *>(filtered);
    const size_t pbytes = (size_t)g->n_angles * n_rows * g->n_det * dtype_size(proj_t);
    const size_t fbytes = (size_t)n_slices * g->n_angles * g->n_det * dtype_size(filtered_t);
    if (pb < fb + fbytes && fb < pb + pbytes) return XCT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    EntryRef ft, taps;
    if (int rc = filter_tables(g->n_det, window, g->det_pitch, s, &ft)) return rc;
    if (radius > 0)
        if (int rc = blur_taps(blur_sigma, radius, s, &taps)) return rc;
    FilterArgs a{};
    a.in = proj;
    a.out = filtered;
    a.tw = ft->table<float2>(0);
    a.H = ft->table<float>(1);
    a.rows = (int64_t)n_slices * g->n_angles;
    a.nc = g->n_det;
    a.L = ft->L;
    a.log2L = ft->lg;
    a.pre.dark = dark;
    a.pre.flat = flat;
    a.pre.taps = taps ? taps->table<float>(0) : nullptr;
    a.pre.radius = radius;
    a.pre.n_rows = n_rows;
    a.pre.row_begin = row_begin;
    a.pre.n_angles = g->n_angles;
    a.pre.floor = floor;
    hipError_t e = launch_front_end_filter(a, proj_t, filtered_t, s);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

// Back-projection of one slab (all entry points but the batch).
static int backproject_one(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
                           void *image, float scale, int32_t accumulate, int out_u16, float code_a,
                           float code_b, hipStream_t s)
{
    BPJob j;
    j.g = g;
    j.n_slices = n_slices;
    j.sino = sino;
    j.image = image;
    j.scale = scale;
    j.accumulate = accumulate ? 1 : 0;
    j.path = choose_path(g);
    j.out_u16 = out_u16;
    j.code_a = code_a;
    j.code_b = code_b;
    if (int rc = geo_tables(g, s, &j.t)) return rc;
    return launch_bp_jobs({j}, sino_t, nullptr, nullptr, s);
}

int xct_backproject(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
                    float *image, float scale, int32_t accumulate, xct_stream stream)
{
    if (int rc = check_geometry(g, true)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (!sino || !image) return XCT_EINVAL;
    if (!dtype_ok(sino_t)) return XCT_EDTYPE;
    if (!std::isfinite(scale)) return XCT_EINVAL;
    return backproject_one(g, n_slices, sino, sino_t, image, scale, accumulate, 0, 0.0f, 0.0f,
                           (hipStream_t)stream);
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
    return backproject_one(g, n_slices, sino, sino_t, image, scale, 0, 1, a32, b32,
                           (hipStream_t)stream);
}

// P = (pixel^2 / pitch) A, the projector of the least-squares problem.
static double projector_scale(const xct_geometry *g) { return g->pixel_size * g->pixel_size / g->det_pitch; }

}  // extern "C"

// sino = (base ? base : accumulate ? sino : 0) + alpha P image.
static int forward_project(const xct_geometry *g, int32_t n_slices, const float *image, const float *base,
                           float *sino, float alpha, int32_t accumulate, xct_stream stream)
{
    if (int rc = check_geometry(g, true)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (!image || !sino) return XCT_EINVAL;
    if (!std::isfinite(alpha)) return XCT_EINVAL;
    if (n_slices > 65535) return XCT_ETOOBIG;
    hipStream_t s = (hipStream_t)stream;
    EntryRef t;
    if (int rc = fp_tables(g, s, &t)) return rc;
    FPArgs a{};
    a.image = image;
    a.sino = sino;
    a.base = base;
    a.ang = t->table<FPAngle>(0);
    a.blocks = t->table<FPBlock>(1);
    a.n_blocks = t->n_blocks;
    a.bin_blocks = (g->n_det + kFPBins - 1) / kFPBins;
    // four slices per workgroup share coordinates and weights; a call with
    // one or two slices keeps one per workgroup
    const int sl = (n_slices >= 3 && t->fp_four) ? 4 : 1;
    // one workgroup per (slice group, bin block, angle block), indexed in 32 bits
    if ((int64_t)a.n_blocks * a.bin_blocks * ((n_slices + sl - 1) / sl) >= ((int64_t)1 << 31)) return XCT_ETOOBIG;
    a.scale = (float)((double)alpha * projector_scale(g));
    a.accumulate = accumulate ? 1 : 0;
    a.n_angles = g->n_angles;
    a.n_det = g->n_det;
    a.nx = g->nx;
    a.ny = g->ny;
    a.n_slices = n_slices;
    if (sl == 1) {
        const hipError_t e = launch_forward(a, 1, s);
        return e == hipSuccess ? XCT_OK : hip_fail(e);
    }
    // Four slices per workgroup read four-slice copies of the image and of
    // its transpose, made chunk by chunk of slice groups in stream-ordered
    // memory (kQuadBytes, or one group when a group needs more).
    const int64_t plane = (int64_t)g->nx * g->ny;
    const int64_t group_bytes = 2 * plane * (int64_t)sizeof(float4);
    const int64_t groups = (n_slices + 3) / 4;
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>(groups, kQuadBytes / group_bytes));
    keep_stream_pool();
    void *buf = nullptr;
    hipError_t e = hipMallocAsync(&buf, (size_t)(per * group_bytes), s);
    if (e != hipSuccess) return hip_fail(e);
    float4 *quad = static_cast<float4 *>(buf), *quad_t = quad + per * plane;
    for (int64_t g0 = 0; g0 < groups && e == hipSuccess; g0 += per) {
        const int64_t z = 4 * g0;
        const int ns = (int)std::min<int64_t>(n_slices - z, 4 * per);
        e = launch_forward_quads(image + z * plane, ns, g->nx, g->ny, quad, quad_t, s);
        if (e != hipSuccess) break;
        FPArgs c = a;
        c.image = image + z * plane;
        c.sino = sino + z * (int64_t)g->n_angles * g->n_det;
        if (base) c.base = base + z * (int64_t)g->n_angles * g->n_det;
        c.n_slices = ns;
        c.quad = quad;
        c.quad_t = quad_t;
        e = launch_forward(c, 4, s);
    }
    const hipError_t f = hipFreeAsync(buf, s);
    if (e == hipSuccess) e = f;
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

extern "C" {

int xct_forward_project(const xct_geometry *g, int32_t n_slices, const float *image, float *sino,
                        float alpha, int32_t accumulate, xct_stream stream)
{
    return forward_project(g, n_slices, image, nullptr, sino, alpha, accumulate, stream);
}

int xct_forward_residual(const xct_geometry *g, int32_t n_slices, const float *image, const float *y,
                         float *r, float alpha, xct_stream stream)
{
    if (!y) return XCT_EINVAL;
    return forward_project(g, n_slices, image, y, r, alpha, 0, stream);
}

int xct_project_adjoint(const xct_geometry *g, int32_t n_slices, const float *sino, float *image,
                        float alpha, int32_t accumulate, xct_stream stream)
{
    if (int rc = check_geometry(g, true)) return rc;
    if (int rc = check_slices(g, n_slices)) return rc;
    if (!sino || !image) return XCT_EINVAL;
    if (!std::isfinite(alpha)) return XCT_EINVAL;
    return backproject_one(g, n_slices, sino, XCT_F32, image, (float)((double)alpha * projector_scale(g)),
                           accumulate, 0, 0.0f, 0.0f, (hipStream_t)stream);
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

// Workspace layout of xct_fbp_batch: 256 bytes of work counters (kXcds per
// launch group), the slab descriptor table, then the filtered rows of every
// slab, each region 256-byte aligned.
static size_t table_bytes(int32_t n_slabs) { return align256(sizeof(BPSlab) * (size_t)n_slabs); }

size_t xct_fbp_workspace_bytes(const xct_slab *slabs, int32_t n_slabs, int32_t filtered_t)
{
    if (check_slabs(slabs, n_slabs, false) || !dtype_ok(filtered_t)) return 0;
    size_t bytes = 256 + table_bytes(n_slabs);
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
    static_assert(5 * kXcds * sizeof(unsigned int) <= 256, "work counters exceed their region");
    if (int rc = check_slabs(slabs, n_slabs, true)) return rc;
    if (!dtype_ok(sino_t) || !dtype_ok(filtered_t)) return XCT_EDTYPE;
    if (window < XCT_RAM_LAK || window > XCT_HANN) return XCT_EDTYPE;
    const size_t need = xct_fbp_workspace_bytes(slabs, n_slabs, filtered_t);
    if (!workspace || ((uintptr_t)workspace & 255) || workspace_bytes < need) return XCT_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;

    char *ws = static_cast<char *>(workspace);
    unsigned int *counters = reinterpret_cast<unsigned int *>(ws);
    BPSlab *table = reinterpret_cast<BPSlab *>(ws + 256);
    size_t off = 256 + table_bytes(n_slabs);
    // Launch groups: the generic kernel; the mirror and the symmetric kernel,
    // each with one slice per item (single-slice slabs) or two.  A slab takes
    // the kernel variant a call with that slab alone takes, so the images
    // equal separate calls bit for bit.
    enum { kGroupGeneric = 0, kGroupMirror1, kGroupMirror2, kGroupSym1, kGroupSym2, kGroups };
    std::vector<BPJob> groups[kGroups];
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
        if (int rc = geo_tables(g, s, &j.t)) return rc;
        const int two = j.n_slices >= 2;
        const int grp = j.path == kPathGeneric  ? kGroupGeneric
                        : j.path == kPathMirror ? (two ? kGroupMirror2 : kGroupMirror1)
                                                : (two ? kGroupSym2 : kGroupSym1);
        groups[grp].push_back(j);
    }
    hipError_t e = launch_fill_u32(counters, kGroups * kXcds, 0u, s);
    if (e != hipSuccess) return hip_fail(e);
    // each group reads its descriptors from its own part of the table
    BPSlab *group_table[kGroups];
    size_t first = 0;
    for (int grp = kGroups - 1; grp >= 0; --grp) {
        group_table[grp] = table + first;
        first += groups[grp].size();
    }
    for (int grp = kGroups - 1; grp >= 0; --grp)
        if (int rc = launch_bp_jobs(groups[grp], filtered_t, counters + grp * kXcds, group_table[grp], s))
            return rc;
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

int xct_dot_f64_noalloc(const float *a, const float *b, int64_t n, double *result, xct_stream stream)
{
    if (!a || !b || !result || n <= 0) return XCT_EINVAL;
    const int nb = reduce_blocks(n);
    if (nb > reduce_scratch_doubles()) return XCT_ETOOBIG;  // cannot happen: the partial count is capped
    double *partials = nullptr;
    hipError_t e = reduce_scratch(&partials);
    if (e != hipSuccess) return hip_fail(e);
    e = launch_reduce(a, b, n, result, partials, nb, 0, (hipStream_t)stream);
    return e == hipSuccess ? XCT_OK : hip_fail(e);
}

}  // extern "C"

// Compute units of the current device (cached per device).
int xct::device_cus()
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
