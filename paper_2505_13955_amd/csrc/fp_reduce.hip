// Forward projector (transpose of the back-projector) and FP64 reductions.
//
// Forward projector, gather form: bin n of angle k sums the pixels whose hat
// weight K(u - n) is non-zero,
//   (P x)[k][n] = scale sum_{v,w} x(v, w) max(0, 1 - |A v + B w + u0 - n|),
// where w is the image axis the rays are walked along (rows when |cos| >=
// |sin|, else columns) and v the other, so |A| >= |B| and along each walk step
// a bin's strip crosses at most floor(2/|A|) + 1 pixels, centred on
//   v*(n, w) = (n - u0 - B w) / A.
// A workgroup takes one block of up to 16 consecutive angles that share the
// walk axis and one block of 256 bins; a thread takes one angle and 16 bins
// four apart (16 angles x 4 interleaved bin groups per wavefront).  It walks the
// image a few steps at a time: it stages into LDS, with coalesced reads, the
// rectangle of pixels those strips can touch (zeros outside the image), then
// every thread adds its taps for its 16 bins, and at the end the results go
// out through LDS so that the stores run along bins.  Four slices per
// workgroup read their pixels from a copy of the image with the four slices'
// values side by side, and blocks walking columns from its transpose, so that
// a stage is read along image rows one 16-byte pixel per load.  Each XCD takes a
// contiguous run of (slice group, bin block, angle block) triples, angle
// blocks fastest, so that the workgroups sharing an L2 stage overlapping
// rectangles of the same slices.  Per stage a thread
// anchors its first bin's crossing in FP64 and keeps an integer index plus an
// FP32 offset below 64/|A| + the staged rows' count, so the hat weights
// carry rounding of the order of 2^-17 pixel.  Fixed summation order: the
// output is deterministic.
//
// Reductions: a fixed grid of workgroups accumulates FP64 partial sums
// (wavefront shuffles, then LDS), and one workgroup sums the partials in a
// fixed order, so results are reproducible bit for bit.
#include <cmath>
#include <mutex>

#include "xct_internal.h"

namespace xct {

// ---------------------------------------------------------------- forward projector

// SL slices per workgroup: the slices of one call share the geometry, so one
// thread's crossings, tap indices and hat weights serve SL slices; the staged
// pixels hold SL values (float4 for four slices).
template <int SL> struct FPVec;
template <> struct FPVec<1> {
    typedef float T;
    static __device__ __forceinline__ T pack(const float *x) { return x[0]; }
    static __device__ __forceinline__ float get(const T &v, int) { return v; }
    static __device__ __forceinline__ T zero() { return 0.0f; }
    static __device__ __forceinline__ T fma(float w, const T &x, const T &s) { return fmaf(w, x, s); }
};
template <> struct FPVec<4> {
    typedef float4 T;
    static __device__ __forceinline__ T pack(const float *x) { return make_float4(x[0], x[1], x[2], x[3]); }
    static __device__ __forceinline__ float get(const T &v, int i)
    {
        return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
    }
    static __device__ __forceinline__ T zero() { return make_float4(0.0f, 0.0f, 0.0f, 0.0f); }
    static __device__ __forceinline__ T fma(float w, const T &x, const T &s)
    {
        return make_float4(fmaf(w, x.x, s.x), fmaf(w, x.y, s.y), fmaf(w, x.z, s.z), fmaf(w, x.w, s.w));
    }
};

// Lanes of a wavefront: 16 angles of the block x 4 bin groups; group g of
// wavefront v takes bins 64 v + g + 4 b, b < 16, of the block, and a thread
// accumulates its angle's 16 bins for SL slices.  Lane 4 q + g takes angle
// q and group g, so each 16 lanes that a 16-byte LDS read serves together
// hold four neighbouring angles at four adjacent bins, whose taps lie within
// a few entries of each other (often at the same address) and so on distinct
// banks.  With the 16 angles of one bin in those 16 lanes, the angles' taps
// spread past 16 entries (the same banks) toward the image edges: 17 times
// the bank-conflict cycles.  With groups of 16 consecutive bins the groups'
// taps sat about 16 entries apart, and the kernel ran 8 % slower.
template <int SL>
__global__ __launch_bounds__(kFPBins, 4) void fp_tile_kernel(FPArgs a)
{
    typedef FPVec<SL> V;
    typedef typename V::T VT;
    constexpr int kStageBatch = SL == 1 ? 8 : 4;  // staged pixels in flight per thread
    constexpr int kBinsPerThread = 16;
    constexpr int kOutPitch = kFPBins + 1;        // LDS floats per angle in the output transpose
    static_assert(kFPAngles == 16 && kFPBins == 256, "lane layout: 16 angles x 4 bin groups x 4 wavefronts");
    static_assert(kFPAngles * kOutPitch <= kFPLdsFloats, "output transpose fits the staging buffer");
    __shared__ VT tile[kFPLdsFloats / SL];
    __shared__ int2 range[2];  // per stage (first staged cross index, staged width), two in turn
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 2;                       // angle of the block
    // workgroup i of a launch runs on XCD i mod 8: give each XCD a
    // contiguous run of (slice group, bin block, angle block) triples, angle
    // block fastest, so the workgroups of one XCD stage overlapping pixels
    const int n_wg = (int)gridDim.x, xcd = (int)blockIdx.x & 7, jx = (int)blockIdx.x >> 3;
    const int qx = n_wg >> 3, rx = n_wg & 7;
    const int wg = a.block_base + xcd * qx + min(xcd, rx) + jx;
    const int blk = wg % a.n_blocks;
    const int tb = wg / a.n_blocks;
    const int bb = tb % a.bin_blocks;
    const int z0 = (tb / a.bin_blocks) * SL;
    const int nsl = min(SL, a.n_slices - z0);  // slices present in this group
    const FPBlock B = a.blocks[blk];
    const int walk = B.walk, count = B.count, k0 = B.k0;
    const int nv = walk ? a.ny : a.nx, nw = walk ? a.nx : a.ny;
    const int n0 = bb * kFPBins;
    const int n1 = n0 + kFPBins - 1;  // the plan sizes stages for whole bin blocks
    const int nb = n0 + wave * 64 + (lane & 3);   // this thread's first bin; its bins are nb + 4 b
    const int64_t plane = (int64_t)a.nx * a.ny;
    const float *img = a.image + (int64_t)z0 * plane;
    // four slices: this group's pixels, read along the walk steps' rows
    const float4 *quad = SL == 4 ? (walk ? a.quad_t : a.quad) + (int64_t)(z0 >> 2) * plane : nullptr;
    const int quad_ld = walk ? a.ny : a.nx;
    const int rows = B.rows[SL == 4 ? 1 : 0], pitch = B.pitch[SL == 4 ? 1 : 0];
    const bool on = q < count;
    const FPAngle p = a.ang[k0 + (on ? q : 0)];
    const float invA = (float)p.invA;
    const bool three = p.taps <= 3 && p.absA <= 1.0f;  // hat two to three pixels wide
    const float c1 = 1.0f - p.hw, c3 = fmaf(-2.0f, p.absA, 2.0f);

    VT acc[kBinsPerThread];
#pragma unroll
    for (int b = 0; b < kBinsPerThread; ++b) acc[b] = V::zero();

    // Cross range of the block's strips over the stage at w0, formed by
    // wavefront 0 into one of two slots: v* is linear in (n, w), so its
    // extremes sit at the corners.
    auto plan_range = [&](int w0, int slot) {
        if (tid < 64) {
            const int rc = min(rows, nw - w0);
            double lo = 1e300, hi = -1e300;
            if (tid < 4 * count) {
                const FPAngle pc = a.ang[k0 + (tid >> 2)];
                const double nn = (tid & 1) ? n1 : n0;
                const double ww = (tid & 2) ? w0 + rc - 1 : w0;
                const double vs = (nn - pc.u0 - pc.B * ww) * pc.invA;
                const double h = 1.0 / fabs(pc.A);
                lo = vs - h;
                hi = vs + h;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                lo = fmin(lo, __shfl_xor(lo, off, 64));
                hi = fmax(hi, __shfl_xor(hi, off, 64));
            }
            if (tid == 0) {
                const int vlo = (int)floor(lo) - 1;
                const int vhi = (int)ceil(hi) + 1;
                range[slot] = make_int2(vlo, min(vhi - vlo + 2, pitch));
            }
        }
    };

    // Stages in turn: the next stage's cross range is formed while the
    // current stage is added up, so a stage takes two barriers.
    plan_range(0, 0);
    __syncthreads();
    for (int s = 0, w0 = 0; w0 < nw; ++s, w0 += rows) {
        const int rc = min(rows, nw - w0);
        const int vlo = range[s & 1].x, width = range[s & 1].y;
        const bool stage_on = vlo + width > 0 && vlo < nv;  // the strips reach the image here
        if (stage_on) {
            // Stage walk steps w0 .. w0+rc-1, cross indices vlo .. vlo+width-1,
            // as a flat range of pixels, several in flight per thread.  Four
            // slices and single slices walking rows read consecutive pixels
            // along a row (of the transposed copy when walking columns); a
            // single slice walking columns reads `rows` consecutive columns of
            // one image row together.
            // (f + 1/2) / width in FP32 recovers the staged row of pixel f
            // exactly: the quotient is below 16, its rounding error below 2^-19,
            // and its distance to an integer at least 1/(2 width) >= 2^-14; and
            // (f + 1/2) / rows its column: the quotient is below 2^13, its
            // rounding error below 2^-10, its distance to an integer at least
            // 1/(2 rows) >= 2^-5.
            {
                const bool by_rows = SL == 4 || walk == 0;
                const int total = by_rows ? width * rc : width * rows;
                const float invw = 1.0f / (float)width, invr = 1.0f / (float)rows;
                for (int fb = 0; fb < total; fb += kStageBatch * kFPBins) {
                    VT val[kStageBatch];
                    int dst[kStageBatch];
#pragma unroll
                    for (int i = 0; i < kStageBatch; ++i) {
                        const int f = fb + i * kFPBins + tid;
                        int r, c;
                        if (by_rows) {
                            r = (int)(((float)f + 0.5f) * invw);
                            c = f - r * width;
                        } else {
                            c = (int)(((float)f + 0.5f) * invr);
                            r = f - c * rows;
                        }
                        const int v = vlo + c;
                        const bool in = f < total && r < rc && v >= 0 && v < nv;
                        if constexpr (SL == 4) {
                            val[i] = in ? quad[(int64_t)(w0 + r) * quad_ld + v] : V::zero();
                        } else {
                            float x = 0.0f;
                            if (in) x = img[walk ? (int64_t)v * a.nx + w0 + r : (int64_t)(w0 + r) * a.nx + v];
                            val[i] = x;
                        }
                        dst[i] = f < total ? r * pitch + c : -1;
                    }
#pragma unroll
                    for (int i = 0; i < kStageBatch; ++i)
                        if (dst[i] >= 0) tile[dst[i]] = val[i];
                }
            }
        }
        __syncthreads();  // the stage is in tile; every wavefront has read its range
        // wavefront 0 forms the next stage's range first, so that its
        // latency hides behind its own taps rather than delaying the barrier
        if (w0 + rows < nw) plan_range(w0 + rows, (s + 1) & 1);
        if (stage_on) {
            // This thread's crossings: v*(nb + 4b, w0 + r) - vlo = rel0 + 4b/A + r dv,
            // anchored once per stage in FP64 (integer part bi0, FP32 fraction f00)
            // so that the FP32 offsets stay below 64/|A| + rows (~2^-17 pixel).
            const double rel0 = ((double)nb - p.u0 - p.B * (double)w0) * p.invA - (double)vlo;
            const int bi0 = (int)floor(rel0);
            const float f00 = (float)(rel0 - (double)bi0);
            bool any_hit;
            {
                // skip the stage when no strip of the wavefront reaches the image
                const float e0 = f00 + (float)bi0, eb = 60.0f * invA, er = (float)(rc - 1) * p.dv;
                const float lo = e0 + fminf(eb, 0.0f) + fminf(er, 0.0f);
                const float hi = e0 + fmaxf(eb, 0.0f) + fmaxf(er, 0.0f);
                const bool hits = on && hi + p.hw > (float)(-vlo) - 1.0f && lo - p.hw < (float)(nv - vlo);
                any_hit = __builtin_amdgcn_ballot_w64(hits) != 0;
            }
            if (any_hit) {
                const VT *base = tile + bi0;
                if (three) {
                    // taps at the first pixel inside the hat's left edge e =
                    // crossing - 1/|A| and the next two; with s = ceil(e) - e in
                    // [0, 1) the weights 1 - |A| |pixel - crossing| are |A| s,
                    // 1 - |A| |s + 1 - 1/|A||, and max(2 - 2|A| - |A| s, 0) (the
                    // first never negative, the middle one never clamped)
                    for (int r = 0; r < rc; ++r) {
                        const float er = fmaf((float)r, p.dv, f00) - p.hw;
                        const VT *row = base + r * pitch;
                        // the taps of bin b + 1 are read before bin b's are added
                        VT x[2][3];
                        float w[2][3];
                        auto fetch = [&](int b, VT (&xx)[3], float (&ww)[3]) {
                            const float e = fmaf((float)(4 * b), invA, er);
                            const float vl = ceilf(e);
                            const float sd = vl - e;
                            const VT *src = row + (int)vl;
                            xx[0] = src[0];
                            xx[1] = src[1];
                            xx[2] = src[2];
                            ww[0] = p.absA * sd;
                            ww[1] = fmaf(-p.absA, fabsf(sd + c1), 1.0f);
                            ww[2] = fmaxf(fmaf(-p.absA, sd, c3), 0.0f);
                        };
                        fetch(0, x[0], w[0]);
#pragma unroll
                        for (int b = 0; b < kBinsPerThread; ++b) {
                            if (b + 1 < kBinsPerThread) fetch(b + 1, x[(b + 1) & 1], w[(b + 1) & 1]);
                            acc[b] = V::fma(w[b & 1][0], x[b & 1][0], acc[b]);
                            acc[b] = V::fma(w[b & 1][1], x[b & 1][1], acc[b]);
                            acc[b] = V::fma(w[b & 1][2], x[b & 1][2], acc[b]);
                        }
                    }
                } else {
                    for (int r = 0; r < rc; ++r) {
                        const float vr = fmaf((float)r, p.dv, f00);
                        const VT *row = base + r * pitch;
#pragma unroll
                        for (int b = 0; b < kBinsPerThread; ++b) {
                            const float vloc = fmaf((float)(4 * b), invA, vr);
                            const float vl = ceilf(vloc - p.hw);
                            const float t = vl - vloc;
                            const VT *src = row + (int)vl;
                            for (int m = 0; m < p.taps; ++m) {
                                const float wgt = fmaxf(fmaf(-p.absA, fabsf(t + (float)m), 1.0f), 0.0f);
                                acc[b] = V::fma(wgt, src[m], acc[b]);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();  // the stage's readers are done with tile; the next range is known
    }

    // Output through LDS, one slice at a time, so that each wavefront stores
    // whole runs of consecutive bins: [angle][bin] with a pitch of 257 floats
    // (the 16 angles x 4 bin groups of a write meet distinct banks).
    float *out_lds = reinterpret_cast<float *>(tile);
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
        if (sl >= nsl) break;
        __syncthreads();
#pragma unroll
        for (int b = 0; b < kBinsPerThread; ++b)
            out_lds[q * kOutPitch + (nb - n0) + 4 * b] = V::get(acc[b], sl);
        __syncthreads();
        const int n = n0 + tid;
        if (n < a.n_det) {
            const int64_t row0 = ((int64_t)(z0 + sl) * a.n_angles + k0) * a.n_det + n;
            float *out = a.sino + row0;
            const float *base = a.base ? a.base + row0 : nullptr;
            for (int qq = 0; qq < count; ++qq) {
                const float v = out_lds[qq * kOutPitch + tid];
                float *o = out + (int64_t)qq * a.n_det;
                if (base) *o = fmaf(a.scale, v, base[(int64_t)qq * a.n_det]);
                else *o = a.accumulate ? fmaf(a.scale, v, *o) : a.scale * v;
            }
        }
    }
}

// Four-slice copies of the image for fp_tile_kernel<4>: for slice group g
// (slices 4g .. 4g+3, zero past the last slice) quad[g][y][x] holds the four
// values of pixel (x, y) and quad_t[g][x][y] the same.  32 x 32 pixels per
// workgroup, transposed through LDS.
__global__ __launch_bounds__(256) void fp_quad_kernel(const float *img, int n_slices, int nx, int ny, float4 *quad,
                                                      float4 *quad_t)
{
    __shared__ float4 t[32][33];
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, g = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t plane = (int64_t)nx * ny;
#pragma unroll
    for (int j = ty; j < 32; j += 8) {
        const int x = x0 + tx, y = y0 + j;
        float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (x < nx && y < ny) {
#pragma unroll
            for (int sl = 0; sl < 4; ++sl)
                if (4 * g + sl < n_slices) v[sl] = img[(int64_t)(4 * g + sl) * plane + (int64_t)y * nx + x];
            quad[g * plane + (int64_t)y * nx + x] = make_float4(v[0], v[1], v[2], v[3]);
        }
        t[j][tx] = make_float4(v[0], v[1], v[2], v[3]);
    }
    __syncthreads();
#pragma unroll
    for (int j = ty; j < 32; j += 8) {
        const int x = x0 + j, y = y0 + tx;
        if (x < nx && y < ny) quad_t[g * plane + (int64_t)x * ny + y] = t[tx][j];
    }
}

hipError_t launch_forward_quads(const float *image, int n_slices, int nx, int ny, float4 *quad, float4 *quad_t,
                                hipStream_t s)
{
    (void)hipGetLastError();
    const dim3 grid((unsigned)((nx + 31) / 32), (unsigned)((ny + 31) / 32), (unsigned)((n_slices + 3) / 4));
    hipLaunchKernelGGL(fp_quad_kernel, grid, dim3(256), 0, s, image, n_slices, nx, ny, quad, quad_t);
    return hipGetLastError();
}

hipError_t launch_forward(const FPArgs &a, int sl, hipStream_t s)
{
    // one workgroup per (slice group, bin block, angle block) triple, split
    // so that no launch exceeds 2^32 - 1 work-items
    const int64_t total = (int64_t)a.n_blocks * a.bin_blocks * ((a.n_slices + sl - 1) / sl);
    const int64_t max_x = ((((int64_t)1 << 32) - 1) / kFPBins);
    (void)hipGetLastError();
    FPArgs c = a;
    for (int64_t x0 = 0; x0 < total; x0 += max_x) {
        c.block_base = (int32_t)x0;
        dim3 grid((unsigned)(total - x0 < max_x ? total - x0 : max_x));
        if (sl == 4)
            hipLaunchKernelGGL(fp_tile_kernel<4>, grid, dim3(kFPBins), 0, s, c);
        else
            hipLaunchKernelGGL(fp_tile_kernel<1>, grid, dim3(kFPBins), 0, s, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- forward projector plan

namespace {

constexpr double kFPSpread = 64.0;  // largest spread of one block's crossings (pixels)

double vstar(const FPAngle &p, double n, double w) { return (n - p.u0 - p.B * w) * p.invA; }

// Staged width (plus slack) of a block over the bins n0.. n0+255 and walk
// steps w0 .. w0+rows-1, computed as the kernel computes it.
int stage_width(const std::vector<FPAngle> &ang, const FPBlock &b, int n0, int w0, int rows)
{
    double lo = 1e300, hi = -1e300;
    for (int q = 0; q < b.count; ++q) {
        const FPAngle &p = ang[b.k0 + q];
        const double h = 1.0 / std::fabs(p.A);
        for (int c = 0; c < 4; ++c) {
            const double vs = vstar(p, (c & 1) ? n0 + kFPBins - 1 : n0, (c & 2) ? w0 + rows - 1 : w0);
            lo = std::min(lo, vs - h);
            hi = std::max(hi, vs + h);
        }
    }
    return ((int)std::ceil(hi) + 1) - ((int)std::floor(lo) - 1) + 2 + 2;
}

}  // namespace

int fp_plan(const xct_geometry *g, std::vector<FPAngle> &ang, std::vector<FPBlock> &blocks, bool *four)
{
    const double r = g->pixel_size / g->det_pitch;
    const double cx = 0.5 * (g->nx - 1), cy = 0.5 * (g->ny - 1);
    const int np = g->n_angles, nc = g->n_det;
    ang.resize(np);
    std::vector<int> walk(np);
    for (int k = 0; k < np; ++k) {
        const double C = std::cos(g->angles[k]) * r, S = std::sin(g->angles[k]) * r;
        FPAngle &p = ang[k];
        walk[k] = std::fabs(C) >= std::fabs(S) ? 0 : 1;
        p.A = walk[k] ? S : C;
        p.B = walk[k] ? C : S;
        p.u0 = g->center - C * cx - S * cy;
        p.invA = 1.0 / p.A;
        p.dv = (float)(-p.B / p.A);
        p.hw = (float)(1.0 / std::fabs(p.A));
        p.absA = (float)std::fabs(p.A);
        p.taps = (int)std::floor(2.0 / std::fabs(p.A)) + 1;
    }
    // greedy runs of angles: same walk axis, crossings within kFPSpread pixels
    // of each other everywhere (the spread is linear in (n, w): check corners)
    blocks.clear();
    for (int k = 0; k < np;) {
        const int nw = walk[k] ? g->nx : g->ny;
        int cnt = 1;
        while (cnt < kFPAngles && k + cnt < np && walk[k + cnt] == walk[k]) {
            double spread = 0.0;
            for (int c = 0; c < 4; ++c) {
                const double nn = (c & 1) ? nc - 1 : 0, ww = (c & 2) ? nw - 1 : 0;
                double lo = 1e300, hi = -1e300;
                for (int q = 0; q <= cnt; ++q) {
                    const double vs = vstar(ang[k + q], nn, ww);
                    lo = std::min(lo, vs);
                    hi = std::max(hi, vs);
                }
                spread = std::max(spread, hi - lo);
            }
            if (spread > kFPSpread) break;
            ++cnt;
        }
        blocks.push_back(FPBlock{k, cnt, walk[k], 0, {0, 0}, {0, 0}});
        k += cnt;
    }
    // staging shape of each block, for one and for four slices per
    // workgroup: the most walk steps (at most 16) whose widest stage fits
    // kFPLdsFloats.  The width is convex in the stage origin (n0, w0), so its
    // maximum over the launch sits at the extreme origins.  Blocks near an
    // axis stage more steps at a time than diagonal ones, whose strips cross
    // wider rectangles.
    const int last_bin_block = ((nc - 1) / kFPBins) * kFPBins;
    *four = true;
    for (FPBlock &b : blocks) {
        const int nw = b.walk ? g->nx : g->ny;
        for (int f = 0; f < 2; ++f) {
            const int sl = f ? 4 : 1;
            for (int rows = 16; rows >= 1; --rows) {
                const int last_w0 = ((nw - 1) / rows) * rows;
                int need = 0;
                for (int c = 0; c < 4; ++c)
                    need = std::max(need, stage_width(ang, b, (c & 1) ? last_bin_block : 0,
                                                      (c & 2) ? last_w0 : 0, rows));
                const int pitch = need | 1;  // odd: column-walk staging writes hit distinct banks
                if ((int64_t)pitch * rows * sl <= kFPLdsFloats) {
                    b.rows[f] = rows;
                    b.pitch[f] = pitch;
                    break;
                }
            }
        }
        if (b.rows[0] == 0) return XCT_ETOOBIG;
        if (b.rows[1] == 0) *four = false;
    }
    return XCT_OK;
}

// ---------------------------------------------------------------- reductions

constexpr int kRedThreads = 256;
constexpr int kRedMaxBlocks = 1024;

int reduce_blocks(int64_t n)
{
    int64_t b = (n + kRedThreads * 8 - 1) / (kRedThreads * 8);
    return (int)(b < 1 ? 1 : (b > kRedMaxBlocks ? kRedMaxBlocks : b));
}

__device__ __forceinline__ double block_sum(double s)
{
    __shared__ double part[kRedThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedThreads / 64; ++w) t += part[w];
    return t;
}

__global__ __launch_bounds__(kRedThreads) void reduce_partial_kernel(const float *a, const float *b,
                                                                      int64_t n, double *partials,
                                                                      int sqdist)
{
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kRedThreads;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
        const double x = a[i], y = b[i];
        s += sqdist ? (x - y) * (x - y) : x * y;
    }
    const double t = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRedThreads) void reduce_final_kernel(const double *partials, int nb,
                                                                    double *out)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kRedThreads) s += partials[i];
    const double t = block_sum(s);
    if (threadIdx.x == 0) *out = t;
}

hipError_t launch_reduce(const float *a, const float *b, int64_t n, double *result,
                         double *partials, int nblocks, int sqdist, hipStream_t s)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(reduce_partial_kernel, dim3(nblocks), dim3(kRedThreads), 0, s, a, b, n,
                       partials, sqdist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, nblocks,
                       result);
    return hipGetLastError();
}

// Partial sums of the allocation-free dot product (xct_dot_f64_noalloc):
// one array per device, kept until the process ends.  In host code this name
// is not a device address; reduce_scratch() looks up each device's copy with
// hipGetSymbolAddress (once per device, that device current) and the kernels
// take that pointer.
constexpr int kScratchDoubles = kRedMaxBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];
static_assert(kScratchDoubles >= kRedMaxBlocks, "every reduction's partial sums fit the scratch array");

int reduce_scratch_doubles() { return kScratchDoubles; }

hipError_t reduce_scratch(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<double *>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

__global__ void fill_u32_kernel(unsigned int *p, int n, unsigned int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(unsigned int *p, int n, unsigned int v, hipStream_t s)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace xct
