// Windowed ramp filter of sinogram rows (Section IV-B, first step of FBP).
//
// The filter is a linear convolution of each detector row with the spatial
// kernel h_W of the window, zero outside the detector:
//   q[n] = (1/pitch) sum_{m=0}^{N_c-1} h_W[n-m] p[m].
// With the row zero-padded to L >= 2 N_c - 1 and h_W placed circularly, the
// circular convolution of length L equals the linear one on [0, N_c), so the
// kernel computes it as IFFT(FFT(p) * H) with H = DFT_L(h_W) precomputed on
// the host in FP64 (real and even, since h_W is symmetric).
//
// Two rows share one complex transform: z = p0 + i p1.  Because H is real,
// IFFT(FFT(z) H) = q0 + i q1, so one forward and one inverse complex FFT
// filter two rows with no real-FFT pre/post-processing.  The inverse is done
// as conj(FFT(conj(Z H))) with the 1/(L pitch) folded into H.
//
// The whole transform lives in LDS (L <= 16384 complex FP32 = 128 KiB) and
// runs as mixed-radix Stockham passes (radix 4, plus one radix-2 pass when
// log2 L is odd); each pass reads its operands into registers, synchronises,
// and writes the results in place.  Twiddles exp(-2 pi i e / L) come from a
// table computed on the host in FP64.
#include "xct_internal.h"

namespace xct {

template <typename T>
__device__ __forceinline__ float ld_in(const T *p, int64_t i);
template <>
__device__ __forceinline__ float ld_in<float>(const float *p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float ld_in<f16_t>(const f16_t *p, int64_t i) { return (float)p[i]; }
template <>
__device__ __forceinline__ float ld_in<bf16_t>(const bf16_t *p, int64_t i)
{
    return __uint_as_float((uint32_t)p[i].bits << 16);
}
template <>
__device__ __forceinline__ float ld_in<uint16_t>(const uint16_t *p, int64_t i) { return (float)p[i]; }

template <typename T>
__device__ __forceinline__ void st_out(T *p, int64_t i, float v);
template <>
__device__ __forceinline__ void st_out<float>(float *p, int64_t i, float v) { p[i] = v; }
template <>
__device__ __forceinline__ void st_out<f16_t>(f16_t *p, int64_t i, float v) { p[i] = (f16_t)v; }
template <>
__device__ __forceinline__ void st_out<bf16_t>(bf16_t *p, int64_t i, float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        p[i].bits = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);             // round to nearest even
        p[i].bits = (uint16_t)(u >> 16);
    }
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// LDS position of transform element i: bits 0-3 XORed with bits 3-6.  A
// permutation within aligned groups of 128 elements that takes the four-way
// bank conflicts of the span-1 and span-4 passes' strided writes down to at
// most two-way, with no extra LDS.
__device__ __forceinline__ int sw(int i) { return i ^ ((i >> 3) & 15); }

// One radix-2 Stockham pass of span Ns (only as the first pass, Ns = 1).
__device__ __forceinline__ void pass_r2(float2 *z, int L, int Ns, const float2 *tw, int tid, int nt)
{
    float2 v0[8], v1[8];
    const int half = L >> 1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int j = tid + q * nt;
        if (j < half) {
            v0[q] = z[sw(j)];
            v1[q] = z[sw(j + half)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int j = tid + q * nt;
        if (j < half) {
            const int k = j & (Ns - 1);
            const float2 b = (Ns > 1) ? cmul(v1[q], tw[k * (L / (2 * Ns))]) : v1[q];
            const int base = ((j - k) << 1) + k;
            z[sw(base)] = make_float2(v0[q].x + b.x, v0[q].y + b.y);
            z[sw(base + Ns)] = make_float2(v0[q].x - b.x, v0[q].y - b.y);
        }
    }
    __syncthreads();
}

// One radix-4 Stockham pass of span Ns.  The twiddles are fetched before the
// LDS reads and the barrier, so their latency overlaps both.
__device__ __forceinline__ void pass_r4(float2 *z, int L, int Ns, const float2 *tw, int tid, int nt)
{
    float2 v[4][4], w[4][3];
    const int quarter = L >> 2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = tid + q * nt;
        if (Ns > 1 && j < quarter) {
            const int e1 = (j & (Ns - 1)) * (quarter / Ns);
            w[q][0] = tw[e1];
            w[q][1] = tw[2 * e1];
            w[q][2] = tw[3 * e1];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = tid + q * nt;
        if (j < quarter) {
#pragma unroll
            for (int r = 0; r < 4; ++r) v[q][r] = z[sw(j + r * quarter)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = tid + q * nt;
        if (j < quarter) {
            const int k = j & (Ns - 1);
            float2 x0 = v[q][0], x1 = v[q][1], x2 = v[q][2], x3 = v[q][3];
            if (Ns > 1) {
                x1 = cmul(x1, w[q][0]);
                x2 = cmul(x2, w[q][1]);
                x3 = cmul(x3, w[q][2]);
            }
            const float2 a0 = make_float2(x0.x + x2.x, x0.y + x2.y);
            const float2 a1 = make_float2(x0.x - x2.x, x0.y - x2.y);
            const float2 a2 = make_float2(x1.x + x3.x, x1.y + x3.y);
            const float2 a3 = make_float2(x1.y - x3.y, x3.x - x1.x);  // -i (x1 - x3)
            const int base = ((j - k) << 2) + k;
            z[sw(base)] = make_float2(a0.x + a2.x, a0.y + a2.y);
            z[sw(base + Ns)] = make_float2(a1.x + a3.x, a1.y + a3.y);
            z[sw(base + 2 * Ns)] = make_float2(a0.x - a2.x, a0.y - a2.y);
            z[sw(base + 3 * Ns)] = make_float2(a1.x - a3.x, a1.y - a3.y);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void fft_forward(float2 *z, int L, int log2L, const float2 *tw, int tid,
                                            int nt)
{
    int Ns = 1;
    if (log2L & 1) {
        pass_r2(z, L, 1, tw, tid, nt);
        Ns = 2;
    }
    for (; Ns < L; Ns <<= 2) pass_r4(z, L, Ns, tw, tid, nt);
}

// Line integral of one raw detector sample (Beer-Lambert, Section V-A c
// stage 2): -ln((I - D) / (F - D)), both differences clamped below at `floor`.
__device__ __forceinline__ float beer_lambert(float i, float d, float f, float floor)
{
    return -logf(fmaxf(i - d, floor) / fmaxf(f - d, floor));
}

// Front end of a row pair: rows r0, r0 + 1 of the output are detector row
// row_begin + s of projection k (r = s N_p + k), read from the projection
// stack [N_p][n_rows][N_c] with the dark and flat fields of that detector
// row.  The line integrals are blurred along the channels with the sampled
// Gaussian (edge samples replicated) staged in the upper half of z, which is
// zero padding of the transform and holds N_c <= L/2 values.
template <typename TI>
__device__ __forceinline__ void load_front_end(float2 *z, const FilterArgs &a, int64_t r0, bool has1,
                                               int tid, int nt)
{
    const int L = a.L, nc = a.nc;
    const PreArgs &pre = a.pre;
    const TI *src[2];
    const float *drow[2], *frow[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t r = has1 || h == 0 ? r0 + h : r0;
        const int64_t s = r / pre.n_angles, k = r - s * pre.n_angles;
        const int64_t det_row = pre.row_begin + s;
        src[h] = static_cast<const TI *>(a.in) + (k * pre.n_rows + det_row) * nc;
        drow[h] = pre.dark + det_row * nc;
        frow[h] = pre.flat + det_row * nc;
    }
    const int stage = pre.radius > 0 ? (L >> 1) : 0;  // first element of the staged rows
    for (int n = tid; n < nc; n += nt) {
        const float p0 = beer_lambert(ld_in(src[0], n), drow[0][n], frow[0][n], pre.floor);
        const float p1 = has1 ? beer_lambert(ld_in(src[1], n), drow[1][n], frow[1][n], pre.floor) : 0.0f;
        z[sw(stage + n)] = make_float2(p0, p1);
    }
    if (pre.radius > 0) {
        __syncthreads();
        const int R = pre.radius;
        for (int n = tid; n < nc; n += nt) {
            float b0 = 0.0f, b1 = 0.0f;
            for (int m = -R; m <= R; ++m) {
                const float g = pre.taps[m + R];
                const float2 v = z[sw(stage + min(max(n + m, 0), nc - 1))];
                b0 = fmaf(g, v.x, b0);
                b1 = fmaf(g, v.y, b1);
            }
            z[sw(n)] = make_float2(b0, b1);
        }
        __syncthreads();
    }
    for (int n = nc + tid; n < L; n += nt) z[sw(n)] = make_float2(0.0f, 0.0f);
}

template <typename TI, typename TO, bool PRE>
__global__ __launch_bounds__(1024) void filter_kernel(FilterArgs a)
{
    extern __shared__ float2 z[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int L = a.L, nc = a.nc;
    const int64_t r0 = (int64_t)blockIdx.x * 2;
    const bool has1 = r0 + 1 < a.rows;

    if (PRE) {
        load_front_end<TI>(z, a, r0, has1, tid, nt);
    } else {
        // input rows of in_len samples land on output bins in_first.. (a
        // wider, virtual detector for offset scans), optionally weighted
        const int in_len = a.in_len, first = a.in_first;
        const TI *p0 = static_cast<const TI *>(a.in) + r0 * in_len;
        const TI *p1 = p0 + in_len;
        // four elements of each row in flight per thread
        for (int n0 = tid; n0 < L; n0 += 4 * nt) {
            float x0[4], x1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int m = n0 + u * nt - first;
                const bool in = (unsigned)m < (unsigned)in_len;
                const float w = (in && a.weight) ? a.weight[m] : 1.0f;
                x0[u] = in ? w * ld_in(p0, m) : 0.0f;
                x1[u] = (in && has1) ? w * ld_in(p1, m) : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (n0 + u * nt < L) z[sw(n0 + u * nt)] = make_float2(x0[u], x1[u]);
        }
    }
    __syncthreads();
    fft_forward(z, L, a.log2L, a.tw, tid, nt);
    for (int n = tid; n < L; n += nt) {
        const float h = a.H[n];
        const float2 v = z[sw(n)];
        z[sw(n)] = make_float2(v.x * h, -v.y * h);
    }
    __syncthreads();
    fft_forward(z, L, a.log2L, a.tw, tid, nt);

    TO *o0 = static_cast<TO *>(a.out) + r0 * nc;
    TO *o1 = o0 + nc;
    for (int n = tid; n < nc; n += nt) {
        const float2 v = z[sw(n)];
        st_out(o0, n, v.x);
        if (has1) st_out(o1, n, -v.y);
    }
}

template <typename TI, typename TO, bool PRE>
static hipError_t launch_typed(const FilterArgs &a, hipStream_t s)
{
    const int nt = max(64, min(1024, a.L / 16));
    const size_t lds = (size_t)a.L * sizeof(float2);
    (void)hipGetLastError();  // report only what this launch does
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(filter_kernel<TI, TO, PRE>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int64_t pairs = (a.rows + 1) / 2;
    hipLaunchKernelGGL((filter_kernel<TI, TO, PRE>), dim3((unsigned)pairs), dim3(nt), lds, s, a);
    return hipGetLastError();
}

template <typename TI, bool PRE>
static hipError_t launch_out(const FilterArgs &a, int out_t, hipStream_t s)
{
    if (out_t == XCT_F32) return launch_typed<TI, float, PRE>(a, s);
    if (out_t == XCT_F16) return launch_typed<TI, f16_t, PRE>(a, s);
    return launch_typed<TI, bf16_t, PRE>(a, s);
}

hipError_t launch_filter(const FilterArgs &a, int in_t, int out_t, hipStream_t s)
{
    if (in_t == XCT_F32) return launch_out<float, false>(a, out_t, s);
    if (in_t == XCT_F16) return launch_out<f16_t, false>(a, out_t, s);
    return launch_out<bf16_t, false>(a, out_t, s);
}

hipError_t launch_front_end_filter(const FilterArgs &a, int in_t, int out_t, hipStream_t s)
{
    if (in_t == XCT_U16) return launch_out<uint16_t, true>(a, out_t, s);
    return launch_out<float, true>(a, out_t, s);
}

}  // namespace xct
