// Forward projector (transpose of the back-projector) and FP64 reductions.
//
// Forward projector, gather form: one thread per (slice, angle, bin) sums the
// pixels whose hat weight K(u - n) is non-zero for that bin.  For an angle
// whose ray direction is closer to the y axis (|C| >= |S|) the thread walks the
// image rows: in row i the bin's centre line crosses x at column
//   j*(i) = (n - c - y_i S) / C + (N_x - 1)/2,
// which moves by -S/C per row (tracked in FP64), and only the columns within
// 1/|C| of j* carry weight 1 - |j - j*| |C|.  Otherwise the roles of rows and
// columns swap.  No atomics, fixed summation order: the output is
// deterministic and its weights are exactly the back-projector's hat weights.
//
// Reductions: a fixed grid of workgroups accumulates FP64 partial sums
// (wavefront shuffles, then LDS), and one workgroup sums the partials in a
// fixed order, so results are reproducible bit for bit.
#include "xct_internal.h"

namespace xct {

__global__ __launch_bounds__(256) void fp_gather_kernel(FPArgs a)
{
    const int nblk = (a.n_det + 255) >> 8;
    const int k = blockIdx.x / nblk;
    const int n = (blockIdx.x - k * nblk) * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (n >= a.n_det) return;
    const double2 cd = a.csd[k];
    const float *img = a.image + (int64_t)z * a.nx * a.ny;
    const double C = cd.x, S = cd.y;
    float sum = 0.0f;
    if (fabs(C) >= fabs(S)) {
        const double inv = 1.0 / C;
        const double y0 = -0.5 * (a.ny - 1);
        double jr = (n - a.center - y0 * S) * inv + 0.5 * (a.nx - 1);
        const double step = -S * inv;
        const double hw = fabs(inv);
        const float cf = (float)fabs(C);
        const int mmax = (int)floor(2.0 * hw) + 1;
        for (int i = 0; i < a.ny; ++i, jr += step) {
            const double lo = ceil(jr - hw);
            const int jl = (int)lo;
            const float f = (float)(jr - lo);
            const float *row = img + (int64_t)i * a.nx;
            for (int m = 0; m <= mmax; ++m) {
                const int j = jl + m;
                const float w = 1.0f - fabsf(((float)m - f) * cf);
                if (j >= 0 && j < a.nx && w > 0.0f) sum += w * row[j];
            }
        }
    } else {
        const double inv = 1.0 / S;
        const double x0 = -0.5 * (a.nx - 1);
        double ir = (n - a.center - x0 * C) * inv + 0.5 * (a.ny - 1);
        const double step = -C * inv;
        const double hw = fabs(inv);
        const float sf = (float)fabs(S);
        const int mmax = (int)floor(2.0 * hw) + 1;
        for (int j = 0; j < a.nx; ++j, ir += step) {
            const double lo = ceil(ir - hw);
            const int il = (int)lo;
            const float f = (float)(ir - lo);
            for (int m = 0; m <= mmax; ++m) {
                const int i = il + m;
                const float w = 1.0f - fabsf(((float)m - f) * sf);
                if (i >= 0 && i < a.ny && w > 0.0f) sum += w * img[(int64_t)i * a.nx + j];
            }
        }
    }
    float *out = a.sino + ((int64_t)z * a.n_angles + k) * a.n_det + n;
    *out = a.accumulate ? fmaf(a.scale, sum, *out) : a.scale * sum;
}

hipError_t launch_forward(const FPArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)(((a.n_det + 255) / 256) * a.n_angles), a.n_slices);
    (void)hipGetLastError();
    hipLaunchKernelGGL(fp_gather_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
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
