// Windowed ramp filter of sinogram rows (Section IV-B, first step of FBP).
//
// The filter is a linear convolution of each detector row with the spatial
// kernel h_W of the window, zero outside the detector:
//   q[n] = (1/pitch) sum_{m=0}^{N_c-1} h_W[n-m] p[m].
// With the row zero-padded to L >= 2 N_c - 1 and h_W placed circularly, the
// circular convolution of length L equals the linear one on [0, N_c), so the
// kernel computes it as IFFT_L(FFT_L(x) H) with H = DFT_L(h_W) precomputed on
// the host in FP64 (real and even, since h_W is symmetric).
//
// Each row is filtered inside one workgroup.  The real row x of length
// L = 2M is packed as z[n] = x[2n] + i x[2n+1] and transformed with one
// complex FFT of length M;
// a single pass over the bin pairs (k, M - k) recovers the real row's spectrum
//   X[k] = E + W^k O,  X[M-k] = conj(E - W^k O),  W = exp(-2 pi i / L),
//   E = (Z[k] + conj Z[M-k]) / 2,  O = (Z[k] - conj Z[M-k]) / 2i,
// multiplies it by H, and packs Y = H X back into Z'[k] = (Y[k] + conj
// Y[M-k]) + i (Y[k] - conj Y[M-k]) W^-k, whose inverse FFT of length M holds
// the filtered row as y[2n] + i y[2n+1].  The factors 1/2 and 1/M and the
// 1/pitch fold into H / (L pitch).  The inverse is done as the conjugate of
// the forward transform of conj Z'.
//
// Two kernels share this scheme.  Rows with M = L/2 >= 256 (N_c > 128, every
// workload of the paper's sizes) take filter_fused_kernel: three Stockham
// passes with 32 values per thread in registers, the spectrum step fused
// between the last forward pass and its adjoint (four LDS exchanges per row);
// it is described where it is defined.  Shorter rows take
// filter_small_kernel: the transform lives in LDS as mixed-radix Stockham
// passes (a radix-2 or radix-4 lead pass, then radix-16 passes), one LDS pass
// for the spectrum step, and the inverse as the conjugate of the forward
// transform of conj Z'; twiddles come from an eighth-turn copy of the
// exp(-2 pi i e / L) table held in LDS.
#include <type_traits>

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

// LDS position of transform element i: with p = bits 5-8 of i, bits 0-4 are
// XORed with p ^ (p << 1).  A permutation within aligned groups of 32 elements
// (256 bytes, one pass over the 64 banks) under which every read and write of
// the radix-16, radix-4 and radix-2 passes (32 lanes of 8-byte elements at a
// time, transforms of 64 to 16384 points) meets 32 distinct bank pairs; each
// output bit group the pass strides need is an invertible function of the
// bits of p that vary across the lanes.  No extra LDS.
__device__ __forceinline__ int sw(int i)
{
    const int p = (i >> 5) & 15;
    return i ^ p ^ (p << 1);
}

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

// LDS position of twiddle-table entry i: bits 0-3 XORed with bits 5-8, a
// permutation within aligned groups of 32 entries that spreads the table
// reads of the span-32 radix-16 pass (exponents 16 and 64 entries apart
// across the lanes) over the banks; consecutive entries stay conflict-free.
__device__ __forceinline__ int swt(int i) { return i ^ ((i >> 5) & 15); }

// exp(-2 pi i e / L) for 0 <= e < L/4 from the eighth-turn table
// T[e] = exp(-2 pi i e / L), e <= L/8, held in LDS: past an eighth of a turn
// the cosine and sine swap roles.
__device__ __forceinline__ float2 twiddle(const float2 *T, int e, int L)
{
    const bool low = e <= (L >> 3);
    const float2 t = T[swt(low ? e : (L >> 2) - e)];
    return low ? t : make_float2(-t.y, -t.x);
}

// One radix-4 Stockham pass of span Ns over a transform of length L, with
// twiddles from the LDS eighth-turn table T.  The twiddles are read before
// the operands and the barrier.
__device__ __forceinline__ void pass_r4(float2 *z, int L, int Ns, const float2 *T, int tid, int nt)
{
    float2 v[4][4], w[4][1];
    const int quarter = L >> 2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = tid + q * nt;
        if (Ns > 1 && j < quarter) {
            w[q][0] = twiddle(T, (j & (Ns - 1)) * (quarter / Ns), L);
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
                // w^2 and w^3 from w: one table read per butterfly
                const float2 w2 = cmul(w[q][0], w[q][0]);
                x1 = cmul(x1, w[q][0]);
                x2 = cmul(x2, w2);
                x3 = cmul(x3, cmul(w2, w[q][0]));
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

// Forward radix-4 butterfly in registers: (x0, x1, x2, x3) -> its DFT.
__device__ __forceinline__ void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3)
{
    const float2 a0 = make_float2(x0.x + x2.x, x0.y + x2.y);
    const float2 a1 = make_float2(x0.x - x2.x, x0.y - x2.y);
    const float2 a2 = make_float2(x1.x + x3.x, x1.y + x3.y);
    const float2 a3 = make_float2(x1.y - x3.y, x3.x - x1.x);  // -i (x1 - x3)
    x0 = make_float2(a0.x + a2.x, a0.y + a2.y);
    x1 = make_float2(a1.x + a3.x, a1.y + a3.y);
    x2 = make_float2(a0.x - a2.x, a0.y - a2.y);
    x3 = make_float2(a1.x - a3.x, a1.y - a3.y);
}

// One radix-16 Stockham pass of span Ns over a transform of length L (one
// butterfly per thread: L / 16 <= nt).  Operand t of butterfly j is element
// j + t L/16; it is turned by w^t, w = exp(-2 pi i k / (16 Ns)), k = j mod Ns,
// with w and w^4 read from the eighth-turn table and the other powers formed
// by at most three products.  The 16-point DFT runs in registers as four
// 4-point DFTs over t = 4a + b, the factors exp(-2 pi i b s1 / 16), and four
// 4-point DFTs over b; output s1 + 4 s2 goes to element (j - k) 16 + k +
// (s1 + 4 s2) Ns.
__device__ __forceinline__ void pass_r16(float2 *z, int L, int Ns, const float2 *T, int tid, int nt)
{
    const int sixteenth = L >> 4;
    const int j = tid;
    const bool on = j < sixteenth;
    float2 x[16];
    float2 w1 = make_float2(1.0f, 0.0f), w4 = w1;
    const int k = j & (Ns - 1);
    if (on && Ns > 1) {
        const int e = k * (sixteenth / Ns);
        w1 = twiddle(T, e, L);
        w4 = twiddle(T, 4 * e, L);
    }
    if (on) {
#pragma unroll
        for (int t = 0; t < 16; ++t) x[t] = z[sw(j + t * sixteenth)];
    }
    __syncthreads();
    if (on) {
        if (Ns > 1) {
            const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
            const float2 w8 = cmul(w4, w4), w12 = cmul(w8, w4);
            const float2 base[4] = {make_float2(1.0f, 0.0f), w4, w8, w12};
            const float2 fine[3] = {w1, w2, w3};
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (a > 0) x[4 * a] = cmul(x[4 * a], base[a]);
#pragma unroll
                for (int b = 1; b < 4; ++b) x[4 * a + b] = cmul(x[4 * a + b], a > 0 ? cmul(base[a], fine[b - 1]) : fine[b - 1]);
            }
        }
        // 4-point DFTs over a (t = 4a + b): column b, outputs s1 in place of a
#pragma unroll
        for (int b = 0; b < 4; ++b) dft4(x[b], x[4 + b], x[8 + b], x[12 + b]);
        // factors exp(-2 pi i b s1 / 16) on element (s1, b) = x[4 s1 + b]
        const float c1 = 0.92387953251128674f;   // cos(pi/8)
        const float s1c = 0.38268343236508977f;  // sin(pi/8)
        const float r2 = 0.70710678118654752f;   // cos(pi/4)
        const float2 f[10] = {make_float2(1.0f, 0.0f), make_float2(c1, -s1c), make_float2(r2, -r2),
                              make_float2(s1c, -c1), make_float2(0.0f, -1.0f), make_float2(-s1c, -c1),
                              make_float2(-r2, -r2), make_float2(-c1, -s1c), make_float2(-1.0f, 0.0f),
                              make_float2(-c1, s1c)};
#pragma unroll
        for (int s1 = 1; s1 < 4; ++s1)
#pragma unroll
            for (int b = 1; b < 4; ++b)
                x[4 * s1 + b] = b * s1 == 4 ? make_float2(x[4 * s1 + b].y, -x[4 * s1 + b].x)  // times -i
                                            : cmul(x[4 * s1 + b], f[b * s1]);
        // 4-point DFTs over b: row s1, outputs s2
#pragma unroll
        for (int s1 = 0; s1 < 4; ++s1) dft4(x[4 * s1], x[4 * s1 + 1], x[4 * s1 + 2], x[4 * s1 + 3]);
        const int base = ((j - k) << 4) + k;
#pragma unroll
        for (int s1 = 0; s1 < 4; ++s1)
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) z[sw(base + (s1 + 4 * s2) * Ns)] = x[4 * s1 + s2];
    }
    __syncthreads();
}

// Forward FFT of length L = 2^log2L in place; T is the eighth-turn twiddle
// table of length L in LDS.  The factor 2^(log2L mod 4) goes first (radix 2,
// 4, or 2 then 4), the rest in radix-16 passes.
__device__ __forceinline__ void fft_forward(float2 *z, int L, int log2L, const float2 *T, int tid, int nt)
{
    int Ns = 1;
    const int lead = log2L & 3;
    if (lead == 1 || lead == 3) {
        pass_r2(z, L, 1, T, tid, nt);
        Ns = 2;
    }
    if (lead >= 2) {
        pass_r4(z, L, Ns, T, tid, nt);
        Ns <<= 2;
    }
    for (; Ns < L; Ns <<= 4) pass_r16(z, L, Ns, T, tid, nt);
}

// Line integral of one raw detector sample (Beer-Lambert, Section V-A c
// stage 2): -ln((I - D) / (F - D)), both differences clamped below at `floor`.
// The quotient takes the hardware reciprocal (about one ulp) of F - D, which
// floor >= the smallest normal float and the cap at 2^126 keep normal; the
// logarithm is the hardware base-2 logarithm of the quotient taken at least
// 2^-126 (normal), so p <= 126 ln 2 = 87.3 (a transmission of 1e-38).
__device__ __forceinline__ float beer_lambert(float i, float d, float f, float floor)
{
    const float ratio = fmaxf(i - d, floor) * __builtin_amdgcn_rcpf(fminf(fmaxf(f - d, floor), 0x1p126f));
    return -0.69314718056f * __builtin_amdgcn_logf(fmaxf(ratio, 0x1p-126f));
}

// Front end of one row: row r of the output is detector row row_begin + s of
// projection k (r = s N_p + k), read from the projection stack
// [N_p][n_rows][N_c] with the dark and flat fields of that detector row.  The
// line integrals are blurred along the channels with the sampled Gaussian
// (edge samples replicated); the unblurred row is staged as plain floats in
// the upper half of the transform buffer (N_c <= L/2 = M floats), which the
// packed row does not reach before the padding is cleared.
template <typename TI>
__device__ __forceinline__ void load_front_end(float2 *z, const FilterArgs &a, int64_t r, int tid, int nt)
{
    const int L = a.L, M = L >> 1, nc = a.nc;
    const PreArgs &pre = a.pre;
    const int64_t s = r / pre.n_angles, k = r - s * pre.n_angles;
    const int64_t det_row = pre.row_begin + s;
    const TI *src = static_cast<const TI *>(a.in) + (k * pre.n_rows + det_row) * nc;
    const float *drow = pre.dark + det_row * nc, *frow = pre.flat + det_row * nc;
    const int npk = (nc + 1) >> 1;  // packed elements holding the row
    if (pre.radius == 0) {
        for (int n = tid; n < npk; n += nt) {
            const int j = 2 * n;
            const float x0 = beer_lambert(ld_in(src, j), drow[j], frow[j], pre.floor);
            const float x1 = j + 1 < nc ? beer_lambert(ld_in(src, j + 1), drow[j + 1], frow[j + 1], pre.floor)
                                        : 0.0f;
            z[sw(n)] = make_float2(x0, x1);
        }
    } else {
        float *stage = reinterpret_cast<float *>(z) + M;
        for (int j = tid; j < nc; j += nt) stage[j] = beer_lambert(ld_in(src, j), drow[j], frow[j], pre.floor);
        __syncthreads();
        const int R = pre.radius;
        for (int n = tid; n < npk; n += nt) {
            float b[2] = {0.0f, 0.0f};
            if (2 * n >= R && 2 * n + 1 + R < nc) {
                // interior: every tap inside the row
                for (int m = -R; m <= R; ++m) {
                    const float w = pre.taps[m + R];
                    b[0] = fmaf(w, stage[2 * n + m], b[0]);
                    b[1] = fmaf(w, stage[2 * n + 1 + m], b[1]);
                }
            } else {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int j = 2 * n + h;
                    if (j < nc)
                        for (int m = -R; m <= R; ++m)
                            b[h] = fmaf(pre.taps[m + R], stage[min(max(j + m, 0), nc - 1)], b[h]);
                }
            }
            z[sw(n)] = make_float2(b[0], b[1]);
        }
        __syncthreads();  // the staged row is read before the padding overwrites it
    }
    for (int n = npk + tid; n < M; n += nt) z[sw(n)] = make_float2(0.0f, 0.0f);
}

// Bin pairs (k, M - k), k = 0 .. M/2, per thread of the spectrum pass: the
// launch has nt >= M / 16 threads, so M/2 + 1 pairs take at most 9 rounds.
constexpr int kSpecRounds = 9;
// Packed elements per thread of the load phase (M / nt <= 16).
constexpr int kLoadRounds = 16;

template <typename TI, typename TO, bool PRE>
__global__ __launch_bounds__(1024) void filter_small_kernel(FilterArgs a)
{
    extern __shared__ float2 z[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int L = a.L, M = L >> 1, nc = a.nc;
    const int64_t r = a.row_base + blockIdx.x;

    // Every global read of the workgroup is issued here, before the first
    // wait: the row's samples, the twiddle table, and the spectrum pass's
    // factors H[k], H[M-k] and exp(-2 pi i k / L), which stay in registers
    // through the first transform.
    float2 Wk[kSpecRounds];
    float Hk[kSpecRounds], Hm[kSpecRounds];
#pragma unroll
    for (int u = 0; u < kSpecRounds; ++u) {
        const int k = tid + u * nt;
        if (k <= (M >> 1)) {
            Wk[u] = a.tw[k];
            Hk[u] = a.H[k];
            Hm[u] = a.H[M - k];
        }
    }
    // eighth-turn twiddles of the length-M transform, exp(-2 pi i e / M) =
    // the length-L table at 2e, after the packed row
    float2 *T = z + M;
    for (int e = tid; e <= (M >> 3); e += nt) T[swt(e)] = a.tw[2 * e];

    if (PRE) {
        load_front_end<TI>(z, a, r, tid, nt);
    } else {
        // the row's in_len samples land on output bins in_first.. (a wider,
        // virtual detector for offset scans), optionally weighted; packed
        // element n holds bins 2n and 2n + 1
        const int in_len = a.in_len, first = a.in_first;
        const TI *p = static_cast<const TI *>(a.in) + r * in_len;
        float x[kLoadRounds][2];
#pragma unroll
        for (int u = 0; u < kLoadRounds; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int n = tid + u * nt;
                const int m = 2 * n + h - first;
                const bool in = n < M && (unsigned)m < (unsigned)in_len;
                const float w = (in && a.weight) ? a.weight[m] : 1.0f;
                x[u][h] = in ? w * ld_in(p, m) : 0.0f;
            }
#pragma unroll
        for (int u = 0; u < kLoadRounds; ++u)
            if (tid + u * nt < M) z[sw(tid + u * nt)] = make_float2(x[u][0], x[u][1]);
    }
    __syncthreads();
    const int log2M = a.log2L - 1;
    fft_forward(z, M, log2M, T, tid, nt);

    // spectrum of the real row, times H, packed for the inverse (one thread
    // per bin pair; k = 0 and k = M/2 pair with themselves and write the same
    // value twice)
#pragma unroll
    for (int u = 0; u < kSpecRounds; ++u) {
        const int k = tid + u * nt;
        if (k > (M >> 1)) break;
        const int kk = (M - k) & (M - 1);
        const float2 Zk = z[sw(k)], Zm = z[sw(kk)];
        const float2 E = make_float2(0.5f * (Zk.x + Zm.x), 0.5f * (Zk.y - Zm.y));
        const float2 O = make_float2(0.5f * (Zk.y + Zm.y), 0.5f * (Zm.x - Zk.x));
        const float2 W = Wk[u];
        const float2 WO = cmul(W, O);
        const float hk = Hk[u], hm = Hm[u];
        const float2 Yk = make_float2(hk * (E.x + WO.x), hk * (E.y + WO.y));    // H X[k]
        const float2 Ym = make_float2(hm * (E.x - WO.x), -hm * (E.y - WO.y));   // H X[M-k]
        const float2 P = make_float2(Yk.x + Ym.x, Yk.y - Ym.y);                 // Yk + conj Ym
        const float2 Q = cmul(make_float2(Yk.x - Ym.x, Yk.y + Ym.y),            // (Yk - conj Ym) W^-k
                              make_float2(W.x, -W.y));
        const float2 P2 = make_float2(Ym.x + Yk.x, Ym.y - Yk.y);                // Ym + conj Yk
        const float2 Q2 = cmul(make_float2(Ym.x - Yk.x, Ym.y + Yk.y),           // (Ym - conj Yk) W^-(M-k)
                               make_float2(-W.x, -W.y));
        // conjugates of Z' = P + i Q feed the forward transform that inverts
        z[sw(k)] = make_float2(P.x - Q.y, -(P.y + Q.x));
        z[sw(kk)] = make_float2(P2.x - Q2.y, -(P2.y + Q2.x));
    }
    __syncthreads();
    fft_forward(z, M, log2M, T, tid, nt);

    TO *o = static_cast<TO *>(a.out) + r * nc;
    for (int n = tid; 2 * n < nc; n += nt) {
        const float2 v = z[sw(n)];
        st_out(o, 2 * n, v.x);
        if (2 * n + 1 < nc) st_out(o, 2 * n + 1, -v.y);
    }
}

// ============================================================== rows of 512 to 16384 points
//
// For M = L/2 >= 256 the transform runs as three Stockham passes with every
// thread holding 32 complex values in registers (M/32 threads per row,
// 256-thread workgroups of 8192/M rows, 64 KiB of LDS):
//   P1: radix R1 (32 when log2 M is odd, else 16), span 1, straight from the
//       input row (no exchange before it, no twiddles);
//   P2: radix R2 = M/(16 R1) (4 or 16; none when M <= 512), span R1;
//   P3: radix 16, span Ns = M/16.
// The inverse is the adjoint of the forward passes run backwards (P3^H, P2^H,
// P1^H; F^H = M IFFT), and P3^H reads the positions P3 writes, so P3, the
// spectrum step and P3^H run in registers: each thread holds a butterfly j
// of P3 and its mirror Ns - j, whose outputs at k = j + s Ns and
// M - k = (Ns - j) + (15 - s) Ns pair up as the spectrum step needs (thread
// 0 holds the two self-mirrored butterflies 0 and Ns/2).  P1^H writes the
// output row.  Four LDS exchanges per row instead of ten.
//
// LDS index of position p: p with bits 0-4 XORed with a GF(2)-linear function
// of bits 5-12 (columns kSwz), chosen so that the 32 lanes of every 8-byte
// access of every exchange meet 32 distinct bank pairs, except the mirror
// butterflies' accesses of P3, whose 32 lanes straddle two aligned groups
// (two-way conflicts on half of that exchange's accesses).  Because the map
// is linear and every position a thread touches is a per-thread part ORed
// with a compile-time part, an access costs one XOR with a constant plus an
// immediate offset.

constexpr int kSwz[8] = {9, 19, 24, 20, 28, 6, 23, 1};

__host__ __device__ constexpr int swz_hi(int q)
{
    int x = 0;
    for (int b = 0; b < 8; ++b)
        if ((q >> b) & 1) x ^= kSwz[b];
    return x;
}

// LDS index of position p (p < 8192): linear over XOR.
__host__ __device__ constexpr int lpos(int p) { return p ^ swz_hi(p >> 5); }

// Element at position base | c, with sb = 8 lpos(base) (a byte offset) and c
// a compile-time position whose bits are disjoint from base's: one XOR with
// a constant, and the rest of c as the instruction's immediate offset.
__device__ __forceinline__ float2 &lds_at(float2 *z, int sb, int c)
{
    const int x = (lpos(c) & 31) << 3;
    return *reinterpret_cast<float2 *>(reinterpret_cast<char *>(z) + ((sb ^ x) + ((c & ~31) << 3)));
}

// The same value, recomputed rather than held: keeps the compiler from
// carrying a pass's addresses or twiddles in registers to its adjoint.
__device__ __forceinline__ int opaque_i(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj_mul(float2 a, float2 b)  // a conj(b)
{
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// multiply by -i (forward) or +i (adjoint)
template <bool INV>
__device__ __forceinline__ float2 rot_i(float2 x)
{
    return INV ? make_float2(-x.y, x.x) : make_float2(x.y, -x.x);
}

// cos and sin of 2 pi e / 64, e = 0 .. 63 (quarter turns exact)
constexpr float kCos64[64] = {1.0f, 0.9951847195625305f, 0.9807852506637573f, 0.9569403529167175f, 0.9238795042037964f, 0.8819212913513184f, 0.8314695954322815f, 0.7730104327201843f, 0.7071067690849304f, 0.6343932747840881f, 0.5555702447891235f, 0.4713967442512512f, 0.3826834261417389f, 0.290284663438797f, 0.19509032368659973f, 0.0980171412229538f, 0.0f, -0.0980171412229538f, -0.19509032368659973f, -0.290284663438797f, -0.3826834261417389f, -0.4713967442512512f, -0.5555702447891235f, -0.6343932747840881f, -0.7071067690849304f, -0.7730104327201843f, -0.8314695954322815f, -0.8819212913513184f, -0.9238795042037964f, -0.9569403529167175f, -0.9807852506637573f, -0.9951847195625305f, -1.0f, -0.9951847195625305f, -0.9807852506637573f, -0.9569403529167175f, -0.9238795042037964f, -0.8819212913513184f, -0.8314695954322815f, -0.7730104327201843f, -0.7071067690849304f, -0.6343932747840881f, -0.5555702447891235f, -0.4713967442512512f, -0.3826834261417389f, -0.290284663438797f, -0.19509032368659973f, -0.0980171412229538f, 0.0f, 0.0980171412229538f, 0.19509032368659973f, 0.290284663438797f, 0.3826834261417389f, 0.4713967442512512f, 0.5555702447891235f, 0.6343932747840881f, 0.7071067690849304f, 0.7730104327201843f, 0.8314695954322815f, 0.8819212913513184f, 0.9238795042037964f, 0.9569403529167175f, 0.9807852506637573f, 0.9951847195625305f};
constexpr float kSin64[64] = {0.0f, 0.0980171412229538f, 0.19509032368659973f, 0.290284663438797f, 0.3826834261417389f, 0.4713967442512512f, 0.5555702447891235f, 0.6343932747840881f, 0.7071067690849304f, 0.7730104327201843f, 0.8314695954322815f, 0.8819212913513184f, 0.9238795042037964f, 0.9569403529167175f, 0.9807852506637573f, 0.9951847195625305f, 1.0f, 0.9951847195625305f, 0.9807852506637573f, 0.9569403529167175f, 0.9238795042037964f, 0.8819212913513184f, 0.8314695954322815f, 0.7730104327201843f, 0.7071067690849304f, 0.6343932747840881f, 0.5555702447891235f, 0.4713967442512512f, 0.3826834261417389f, 0.290284663438797f, 0.19509032368659973f, 0.0980171412229538f, 0.0f, -0.0980171412229538f, -0.19509032368659973f, -0.290284663438797f, -0.3826834261417389f, -0.4713967442512512f, -0.5555702447891235f, -0.6343932747840881f, -0.7071067690849304f, -0.7730104327201843f, -0.8314695954322815f, -0.8819212913513184f, -0.9238795042037964f, -0.9569403529167175f, -0.9807852506637573f, -0.9951847195625305f, -1.0f, -0.9951847195625305f, -0.9807852506637573f, -0.9569403529167175f, -0.9238795042037964f, -0.8819212913513184f, -0.8314695954322815f, -0.7730104327201843f, -0.7071067690849304f, -0.6343932747840881f, -0.5555702447891235f, -0.4713967442512512f, -0.3826834261417389f, -0.290284663438797f, -0.19509032368659973f, -0.0980171412229538f};

// exp(-2 pi i e / n) (forward) or its conjugate, n dividing 64
template <bool INV>
__device__ __forceinline__ float2 root(int e, int n)
{
    const int i = (((e % n) + n) % n) * (64 / n);
    return make_float2(kCos64[i], INV ? kSin64[i] : -kSin64[i]);
}

template <bool INV>
__device__ __forceinline__ void bfly4(float2 &x0, float2 &x1, float2 &x2, float2 &x3)
{
    const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = rot_i<INV>(csub(x1, x3));
    x0 = cadd(a0, a2);
    x1 = cadd(a1, a3);
    x2 = csub(a0, a2);
    x3 = csub(a1, a3);
}

// Multiply by the compile-time root exp(-+2 pi i e / n), with the trivial
// quarter turns and the eighth turns done without a full product.
template <bool INV>
__device__ __forceinline__ float2 turn(float2 x, int e, int n)
{
    e %= n;
    if (e == 0) return x;
    if (4 * e == n) return rot_i<INV>(x);
    if (2 * e == n) return make_float2(-x.x, -x.y);
    if (4 * e == 3 * n) return rot_i<!INV>(x);
    const float2 w = root<INV>(e, n);
    return make_float2(x.x * w.x - x.y * w.y, x.x * w.y + x.y * w.x);
}

// DFT of 4, 16 or 32 points in registers (forward: exp(-2 pi i t s / R);
// adjoint: the conjugate).  Input t in x[t]; output s in x[dft_slot<R>(s)].
template <int R>
__host__ __device__ constexpr int dft_slot(int s)
{
    return R == 4 ? s : R == 16 ? 4 * (s & 3) + (s >> 2) : ((s & 1) ? 16 : 0) + 4 * ((s >> 1) & 3) + (s >> 3);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 *x)
{
    if constexpr (R == 4) {
        bfly4<INV>(x[0], x[1], x[2], x[3]);
    } else if constexpr (R == 16) {
        // t = 4 t1 + t2: DFT over t1 per t2, factors w16^(t2 s1), DFT over t2 per s1
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2) bfly4<INV>(x[t2], x[4 + t2], x[8 + t2], x[12 + t2]);
#pragma unroll
        for (int s1 = 1; s1 < 4; ++s1)
#pragma unroll
            for (int t2 = 1; t2 < 4; ++t2) x[4 * s1 + t2] = turn<INV>(x[4 * s1 + t2], s1 * t2, 16);
#pragma unroll
        for (int s1 = 0; s1 < 4; ++s1) bfly4<INV>(x[4 * s1], x[4 * s1 + 1], x[4 * s1 + 2], x[4 * s1 + 3]);
    } else {
        // t = b + 16 a: pairs (b, b + 16), factors w32^(b s1), 16-point DFTs over b
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const float2 u = x[b], v = x[b + 16];
            x[b] = cadd(u, v);
            x[b + 16] = turn<INV>(csub(u, v), b, 32);
        }
        dft<16, INV>(x);
        dft<16, INV>(x + 16);
    }
}

// Powers w^1 .. w^15 of a butterfly's twiddle from w and w^4 (at most three
// products each); p[0] = 1.
__device__ __forceinline__ void powers16(float2 w1, float2 w4, float2 *p)
{
    const float2 one = make_float2(1.0f, 0.0f);
    const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
    const float2 w8 = cmul(w4, w4), w12 = cmul(w8, w4);
    const float2 base[4] = {one, w4, w8, w12}, fine[4] = {one, w1, w2, w3};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) p[4 * a + b] = (a == 0) ? fine[b] : (b == 0) ? base[a] : cmul(base[a], fine[b]);
}

// Spectrum step for the bin pair (k, M - k) of the packed transform Z:
// real-row spectrum X[k] = E + W^k O, X[M-k] = conj(E - W^k O) with
// E = (Z[k] + conj Z[M-k]) / 2, O = (Z[k] - conj Z[M-k]) / 2i, times the
// filter (hk = H[k], hm = H[M-k], scaled by 1 / (L pitch)), repacked as
//   Z'[k]   = P + i Q,  P = Y[k] + conj Y[M-k],  Q = (Y[k] - conj Y[M-k]) W^-k
//   Z'[M-k] = conj P + i conj Q,
// whose adjoint transform F^H Z' is the filtered row (even samples in the
// real parts, odd in the imaginary parts).  w = W^k = exp(-2 pi i k / L).
__device__ __forceinline__ void spectrum_pair(float2 zk, float2 zm, float2 w, float hk, float hm, float2 &ok,
                                              float2 &om)
{
    const float2 E = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 O = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
    const float2 WO = cmul(w, O);
    const float2 Yk = make_float2(hk * (E.x + WO.x), hk * (E.y + WO.y));
    const float2 Ym = make_float2(hm * (E.x - WO.x), -hm * (E.y - WO.y));
    const float2 P = make_float2(Yk.x + Ym.x, Yk.y - Ym.y);
    const float2 Q = cconj_mul(make_float2(Yk.x - Ym.x, Yk.y + Ym.y), w);
    ok = make_float2(P.x - Q.y, P.y + Q.x);
    om = make_float2(P.x + Q.y, Q.x - P.y);
}

// Keep the compiler from merging a recomputation with an earlier value (the
// adjoint passes recompute their twiddle powers instead of holding them).
__device__ __forceinline__ float2 opaque(float2 v)
{
    asm volatile("" : "+v"(v.x), "+v"(v.y));
    return v;
}

// P1 inputs of the filter: element e = T + b TN + t M/R1 of row r holds
// output bins 2e and 2e + 1; the input row's samples land on bins in_first ..
// in_first + in_len - 1 (times `weight` when given), zero elsewhere.  Every
// load reads a valid address (clamped) and the value is selected after, so
// the loads issue back to back without branches.
template <typename TI, bool SHIFTED>
__device__ __forceinline__ float in_bin(const TI *p, const float *weight, int first, int len, int b)
{
    const int m = SHIFTED ? b - first : b;
    const bool in = (unsigned)m < (unsigned)len;
    const int mc = in ? m : 0;
    float v = ld_in(p, mc);
    if (SHIFTED && weight) v *= weight[mc];
    return in ? v : 0.0f;
}

// Both samples of element e in one load (an unshifted row of even length
// from a buffer aligned to two samples: every element is so aligned).
template <typename TI>
__device__ __forceinline__ float2 ld_pair(const TI *p, int e);
template <>
__device__ __forceinline__ float2 ld_pair<float>(const float *p, int e)
{
    return reinterpret_cast<const float2 *>(p)[e];
}
template <>
__device__ __forceinline__ float2 ld_pair<f16_t>(const f16_t *p, int e)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 v = reinterpret_cast<const h2 *>(p)[e];
    return make_float2((float)v.x, (float)v.y);
}
template <>
__device__ __forceinline__ float2 ld_pair<bf16_t>(const bf16_t *p, int e)
{
    const uint32_t u = reinterpret_cast<const uint32_t *>(p)[e];
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}

// MODE 0: unshifted row of even length (pair loads); 1: unshifted; 2:
// shifted and/or weighted.  The row fills at most the first half of the
// packed elements (2e < in_first + in_len <= N_c <= M), so only inputs t <
// R1/2 of each P1 butterfly are read: x[b * (R1/2) + t].
template <int R1, int NB1, int TN, int M, typename TI, int MODE>
__device__ __forceinline__ void load_p1(float2 *x, const FilterArgs &a, int64_t r, int T)
{
    const TI *p = static_cast<const TI *>(a.in) + r * a.in_len;
    const float *w = a.weight;
    const int first = a.in_first, len = a.in_len;
#pragma unroll
    for (int b = 0; b < NB1; ++b)
#pragma unroll
        for (int t = 0; t < R1 / 2; ++t) {
            const int e = T + b * TN + t * (M / R1);
            if constexpr (MODE == 0) {
                const bool in = 2 * e < len;
                const float2 v = ld_pair(p, in ? e : 0);
                x[b * (R1 / 2) + t] = in ? v : make_float2(0.0f, 0.0f);
            } else {
                x[b * (R1 / 2) + t] = make_float2(in_bin<TI, MODE == 2>(p, w, first, len, 2 * e),
                                                  in_bin<TI, MODE == 2>(p, w, first, len, 2 * e + 1));
            }
        }
}

template <int R1, int NB1, int TN, int M, typename TI>
__device__ __forceinline__ void load_p1_t(float2 *x, const FilterArgs &a, int64_t r, int T)
{
    if (a.weight || a.in_first != 0) load_p1<R1, NB1, TN, M, TI, 2>(x, a, r, T);
    else if ((a.in_len & 1) == 0 && reinterpret_cast<uintptr_t>(a.in) % (2 * sizeof(TI)) == 0)
        load_p1<R1, NB1, TN, M, TI, 0>(x, a, r, T);
    else load_p1<R1, NB1, TN, M, TI, 1>(x, a, r, T);
}

template <int R1, int NB1, int TN, int M>
__device__ __forceinline__ void load_p1_any(float2 *x, const FilterArgs &a, int in_t, int64_t r, int T)
{
    if (in_t == XCT_F32) load_p1_t<R1, NB1, TN, M, float>(x, a, r, T);
    else if (in_t == XCT_F16) load_p1_t<R1, NB1, TN, M, f16_t>(x, a, r, T);
    else load_p1_t<R1, NB1, TN, M, bf16_t>(x, a, r, T);
}

// P1^H outputs: element e of the row holds bins 2e (real part) and 2e + 1;
// only outputs t < R1/2 of each butterfly fall on the row (2e < N_c <= M).
// An FP32 row of even length in an 8-byte aligned buffer takes both samples
// in one 8-byte store.
template <int R1, int NB1, int TN, int M, typename TO>
__device__ __forceinline__ void store_p1(const float2 *x, const FilterArgs &a, int64_t r, int T)
{
    TO *o = static_cast<TO *>(a.out) + r * a.nc;
    const int nc = a.nc;
    const bool pairs = sizeof(TO) == 4 && (nc & 1) == 0 && reinterpret_cast<uintptr_t>(a.out) % 8 == 0;
#pragma unroll
    for (int b = 0; b < NB1; ++b)
#pragma unroll
        for (int t = 0; t < R1 / 2; ++t) {
            const int e = T + b * TN + t * (M / R1);
            const float2 v = x[b * R1 + dft_slot<R1>(t)];
            if (pairs) {
                if (2 * e < nc) reinterpret_cast<float2 *>(o)[e] = v;
            } else {
                if (2 * e < nc) st_out(o, 2 * e, v.x);
                if (2 * e + 1 < nc) st_out(o, 2 * e + 1, v.y);
            }
        }
}

// Persistent front end: a raw uint16 row of N_c = 4 n_q counts is read in
// quads (8 bytes); thread T of a row takes quads T + i TN, i < 8 (8 TN = M/4
// quads cover any N_c <= M).  Quads past the row re-read the row's last quad
// (in bounds); those values are never used.
__device__ __forceinline__ float4 quad_f32(uint2 v)
{
    return make_float4((float)(v.x & 0xffffu), (float)(v.x >> 16), (float)(v.y & 0xffffu), (float)(v.y >> 16));
}

template <int TN>
__device__ __forceinline__ void load_raw_quads(uint2 (&q)[8], const FilterArgs &a, int64_t r, int T)
{
    const PreArgs &pre = a.pre;
    const int64_t s = r / pre.n_angles, kp = r - s * pre.n_angles;
    const uint2 *row = reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(a.in) +
                                                       (kp * pre.n_rows + pre.row_begin + s) * a.nc);
    const int last = (a.nc >> 2) - 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = row[min(T + i * TN, last)];
}

// Gaussian blur (taps w[-R..R], edge samples replicated) of a staged row of
// N_c = 4 n_q samples from src into dst, by quads: thread T of the row takes
// quads T + i TN, i < 8.  A quad whose taps stay inside the row reads its
// neighbour quads as 16-byte words; the quads within R samples of an end
// read clamped samples one at a time.  (Blurs of R <= 4 take a path without
// the second buffer, in the kernel.)
template <int TN>
__device__ __forceinline__ void blur_quads(const float *src, float *dst, int nc, int R, const float *w, int T)
{
    const int nq = nc >> 2;
    const int QR = (R + 3) >> 2;  // neighbour quads each side
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    float4 *d4 = reinterpret_cast<float4 *>(dst);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int q = T + i * TN;
        if (q >= nq) continue;
        float o[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (q >= QR && q + QR < nq) {
            for (int j = -QR; j <= QR; ++j) {
                const float4 u = s4[q + j];
                const float v[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int cc = 0; cc < 4; ++cc)
#pragma unroll
                    for (int cp = 0; cp < 4; ++cp) {
                        const int m = 4 * j + cp - cc;
                        if (m >= -R && m <= R) o[cc] = fmaf(w[m + R], v[cp], o[cc]);
                    }
            }
        } else {
            for (int m = -R; m <= R; ++m) {
                const float wm = w[m + R];
#pragma unroll
                for (int c = 0; c < 4; ++c) o[c] = fmaf(wm, src[min(max(4 * q + c + m, 0), nc - 1)], o[c]);
            }
        }
        d4[q] = make_float4(o[0], o[1], o[2], o[3]);
    }
}

// Kernel kinds: the front end (raw projection stack); any row form with one
// workgroup per group of rows; persistent kernels for unshifted, unweighted
// rows of even length in FP32, FP16 or BF16 that keep the next group's
// samples in flight; a persistent front end (uint16 counts, N_c a multiple
// of 4, stack and fields aligned to quads) that keeps the next group's counts
// in flight; and a persistent kernel for FP32 rows of any other form
// (shifted, weighted, odd lengths, element-wise loads).
enum {
    kFrontEnd = 0,
    kRows = 1,
    kPersistF32 = 2,
    kPersistF16 = 3,
    kPersistBF16 = 4,
    kPersistFE16 = 5,
    kPersistAnyF32 = 6
};

template <int LOG2M, int KIND>
__global__ __launch_bounds__(256) void filter_fused_kernel(FilterArgs a, int in_t, int out_t)
{
    constexpr bool FEP = KIND == kPersistFE16;
    constexpr bool PRE = KIND == kFrontEnd || FEP;
    constexpr bool PERSIST = KIND >= kPersistF32;
    constexpr int LMODE = KIND == kPersistAnyF32 ? 2 : 0;  // load form of the persistent row kinds
    typedef typename std::conditional<KIND == kPersistF16, f16_t,
                                      typename std::conditional<KIND == kPersistBF16, bf16_t, float>::type>::type TP;
    constexpr int M = 1 << LOG2M;
    constexpr int R1 = (LOG2M & 1) ? 32 : 16;
    constexpr int H1 = R1 / 2;         // P1 inputs per butterfly that can be non-zero
    constexpr int R2 = (M / 16) / R1;  // 1 (no middle pass), 4 or 16
    constexpr int NB1 = 32 / R1;       // P1 butterflies per thread
    constexpr int NB2 = 32 / R2;       // P2 butterflies per thread
    constexpr int NS = M / 16;         // span of P3
    constexpr int TN = M / 32;         // threads per row
    constexpr int ROWS = 256 / TN;     // rows per workgroup
    static_assert(LOG2M >= 8 && LOG2M <= 13, "fused filter: 256 <= M <= 8192");
    __shared__ __align__(16) float2 z[8192];

    const int tid = threadIdx.x;
    const int rho = tid / TN, T_h = tid % TN;
    const int nc = a.nc;
    const int rb = rho * M;  // the row's positions in LDS
    // groups of ROWS rows; this workgroup takes groups blockIdx.x,
    // blockIdx.x + gridDim.x, ...
    const int64_t groups = (a.rows + ROWS - 1) / ROWS;

    // Row-independent twiddles, read once: butterfly A = T of the last pass,
    // its mirror B, and the middle pass's.
    const int A_h = T_h;
    const int B_h = T_h == 0 ? NS / 2 : NS - T_h;
    const float2 WT_h = a.tw[T_h];                            // W^T, W = exp(-2 pi i / L)
    const float2 w1A_h = a.tw[2 * A_h], w4A_h = a.tw[8 * A_h];  // exp(-2 pi i j / M), its fourth power
    const float2 w1B_h = a.tw[2 * B_h], w4B_h = a.tw[8 * B_h];
    float2 w21_h = make_float2(1.0f, 0.0f), w24_h = w21_h;  // exp(-2 pi i (T mod R1) / (R1 R2)), fourth power
    if constexpr (R2 > 1) {
        w21_h = a.tw[32 * (T_h & (R1 - 1))];
        if constexpr (R2 == 16) w24_h = a.tw[128 * (T_h & (R1 - 1))];
    }

    // The plain filter holds the next group's P1 inputs in xn while the
    // current group is transformed.
    float2 xn[NB1 * H1];
    uint2 rq[8];
    int64_t g = blockIdx.x;
    if constexpr (FEP) {
        const int64_t r = g * ROWS + rho;
        if (g < groups && r < a.rows) load_raw_quads<TN>(rq, a, r, T_h);
    } else if constexpr (PERSIST) {
        const int64_t r = g * ROWS + rho;
        if (g < groups && r < a.rows) load_p1<R1, NB1, TN, M, TP, LMODE>(xn, a, r, T_h);
        else
#pragma unroll
            for (int i = 0; i < NB1 * H1; ++i) xn[i] = make_float2(0.0f, 0.0f);
    }

    auto group = [&](int64_t g) {
        // Values that do not change from group to group pass through opaque
        // copies, so that what is derived from them (addresses, predicates,
        // twiddle powers) is recomputed per group rather than held in
        // registers across the loop.
        const int T = opaque_i(T_h);
        const int A = T;
        const int B = opaque_i(B_h);
        const float2 WT = opaque(WT_h), w1A = opaque(w1A_h), w4A = opaque(w4A_h);
        const float2 w1B = opaque(w1B_h), w4B = opaque(w4B_h), w21 = opaque(w21_h), w24 = opaque(w24_h);
        const int k2 = T & (R1 - 1);  // P2: j mod R1 = T mod R1
        const int64_t r = g * ROWS + rho;
        const bool live = r < a.rows;

        float2 x[32];
        // ---- P1 inputs: butterfly T + b TN reads elements j + t M/R1; those
        // with t >= R1/2 are zero
        if constexpr (PERSIST && !FEP) {
#pragma unroll
            for (int b = 0; b < NB1; ++b)
#pragma unroll
                for (int t = 0; t < R1; ++t) x[b * R1 + t] = t < H1 ? xn[b * H1 + t] : make_float2(0.0f, 0.0f);
        } else if constexpr (!PRE) {
            float2 xl[NB1 * H1];
            if (live) load_p1_any<R1, NB1, TN, M>(xl, a, in_t, r, T);
            else
#pragma unroll
                for (int i = 0; i < NB1 * H1; ++i) xl[i] = make_float2(0.0f, 0.0f);
#pragma unroll
            for (int b = 0; b < NB1; ++b)
#pragma unroll
                for (int t = 0; t < R1; ++t) x[b * R1 + t] = t < H1 ? xl[b * H1 + t] : make_float2(0.0f, 0.0f);
        } else {
            // front end: Beer-Lambert of the row into LDS (plain floats), then
            // the blurred samples of this thread's elements
            const PreArgs &pre = a.pre;
            float *stage = reinterpret_cast<float *>(z + rb);
            if (FEP && live) {
                // the row's raw quads are in rq; its dark and flat quads
                // are read here (the fields stay in L2)
                const int64_t det_row = pre.row_begin + r / pre.n_angles;
                const float4 *d4 = reinterpret_cast<const float4 *>(pre.dark + det_row * nc);
                const float4 *f4 = reinterpret_cast<const float4 *>(pre.flat + det_row * nc);
                const int nq = nc >> 2;
                float4 dk[8], fl[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int q = min(T + i * TN, nq - 1);
                    dk[i] = d4[q];
                    fl[i] = f4[q];
                }
                float4 *st4 = reinterpret_cast<float4 *>(stage);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int q = T + i * TN;
                    const float4 v = quad_f32(rq[i]);
                    if (q < nq)
                        st4[q] = make_float4(beer_lambert(v.x, dk[i].x, fl[i].x, pre.floor),
                                             beer_lambert(v.y, dk[i].y, fl[i].y, pre.floor),
                                             beer_lambert(v.z, dk[i].z, fl[i].z, pre.floor),
                                             beer_lambert(v.w, dk[i].w, fl[i].w, pre.floor));
                }
            } else if (live) {
                const int64_t s = r / pre.n_angles;
                const int64_t kp = r - s * pre.n_angles;
                const int64_t det_row = pre.row_begin + s;
                const int64_t src = (kp * pre.n_rows + det_row) * nc;
                const float *drow = pre.dark + det_row * nc, *frow = pre.flat + det_row * nc;
                // a row has at most M = 32 TN samples: 32 per thread, loads
                // issued eight samples at a time
#pragma unroll
                for (int j0 = 0; j0 < 32; j0 += 8) {
                    float raw[8], dk[8], fl[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int j = T + (j0 + u) * TN;
                        const int jc = j < nc ? j : 0;
                        raw[u] = in_t == XCT_U16 ? (float)static_cast<const uint16_t *>(a.in)[src + jc]
                                                 : static_cast<const float *>(a.in)[src + jc];
                        dk[u] = drow[jc];
                        fl[u] = frow[jc];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int j = T + (j0 + u) * TN;
                        if (j < nc) stage[j] = beer_lambert(raw[u], dk[u], fl[u], pre.floor);
                    }
                }
            }
            __syncthreads();
            const int R = pre.radius;
            const int K = (R + 1) >> 1;  // sample pairs each side of an element
#pragma unroll
            for (int i = 0; i < 32; ++i) x[i] = make_float2(0.0f, 0.0f);
            if constexpr (FEP) {
                const float2 *p2 = reinterpret_cast<const float2 *>(stage);
                if (R == 0) {
#pragma unroll
                    for (int b = 0; b < NB1; ++b)
#pragma unroll
                        for (int t = 0; t < H1; ++t) {
                            const int e = T + b * TN + t * (M / R1);
                            if (live && 2 * e < nc) x[b * R1 + t] = p2[e];
                        }
                } else if (R <= 4) {
                    // taps padded to w[-4..4]: element e (bins 2e, 2e + 1)
                    // reads the sample pairs e - 2 .. e + 2 when they lie in
                    // the row; elements near an end read clamped samples
                    float tk[9];
#pragma unroll
                    for (int m = -4; m <= 4; ++m)
                        tk[m + 4] = (m >= -R && m <= R) ? pre.taps[min(max(m + R, 0), 2 * R)] : 0.0f;
#pragma unroll
                    for (int b = 0; b < NB1; ++b)
#pragma unroll
                        for (int t = 0; t < H1; ++t) {
                            const int e = T + b * TN + t * (M / R1);
                            if (!live || 2 * e >= nc) continue;
                            float o0 = 0.0f, o1 = 0.0f;
                            if (e >= 2 && 2 * e + 5 < nc) {
                                float sm[10];  // samples 2e - 4 .. 2e + 5
#pragma unroll
                                for (int k = 0; k < 5; ++k) {
                                    const float2 v = p2[e - 2 + k];
                                    sm[2 * k] = v.x;
                                    sm[2 * k + 1] = v.y;
                                }
#pragma unroll
                                for (int m = -4; m <= 4; ++m) {
                                    o0 = fmaf(tk[m + 4], sm[4 + m], o0);
                                    o1 = fmaf(tk[m + 4], sm[5 + m], o1);
                                }
                            } else {
                                for (int m = -R; m <= R; ++m) {
                                    const float wm = pre.taps[m + R];
                                    o0 = fmaf(wm, stage[min(max(2 * e + m, 0), nc - 1)], o0);
                                    o1 = fmaf(wm, stage[min(max(2 * e + 1 + m, 0), nc - 1)], o1);
                                }
                            }
                            x[b * R1 + t] = make_float2(o0, o1);
                        }
                } else {
                    // wider blurs: the blurred row into the upper half of
                    // the row's region (N_c <= M floats each), then the
                    // elements' sample pairs
                    if (live) blur_quads<TN>(stage, stage + M, nc, R, pre.taps, T);
                    __syncthreads();
                    const float2 *b2 = reinterpret_cast<const float2 *>(stage + M);
#pragma unroll
                    for (int b = 0; b < NB1; ++b)
#pragma unroll
                        for (int t = 0; t < H1; ++t) {
                            const int e = T + b * TN + t * (M / R1);
                            if (live && 2 * e < nc) x[b * R1 + t] = b2[e];
                        }
                }
            } else if (R == 0) {
#pragma unroll
                for (int b = 0; b < NB1; ++b)
#pragma unroll
                    for (int t = 0; t < H1; ++t) {
                        const int e = T + b * TN + t * (M / R1);
                        if (live && 2 * e < nc)
                            x[b * R1 + t] = make_float2(stage[2 * e], 2 * e + 1 < nc ? stage[2 * e + 1] : 0.0f);
                    }
            } else {
                // Interior elements (every tap inside the row): pairs q_k =
                // (s[2e + 2k], s[2e + 2k + 1]), |k| <= K, cover samples
                // 2e - R .. 2e + 1 + R; bin 2e takes weights w(2k), w(2k + 1),
                // bin 2e + 1 takes w(2k - 1), w(2k) (w zero beyond |m| = R).
                // The weights are uniform: read once per pair offset.
                const float2 *pairs = reinterpret_cast<const float2 *>(stage);
                for (int k = -K; k <= K; ++k) {
                    const int m0 = 2 * k;
                    const float wm = m0 - 1 >= -R ? pre.taps[m0 - 1 + R] : 0.0f;  // m0 - 1 <= R always
                    const float w0 = (m0 >= -R && m0 <= R) ? pre.taps[m0 + R] : 0.0f;
                    const float wp = m0 + 1 <= R ? pre.taps[m0 + 1 + R] : 0.0f;   // m0 + 1 >= -R always
#pragma unroll
                    for (int b = 0; b < NB1; ++b)
#pragma unroll
                        for (int t = 0; t < H1; ++t) {
                            const int e = T + b * TN + t * (M / R1);
                            if (live && e >= K && 2 * e + 1 + 2 * K < nc) {
                                const float2 q = pairs[e + k];
                                float2 &v = x[b * R1 + t];
                                v.x = fmaf(w0, q.x, fmaf(wp, q.y, v.x));
                                v.y = fmaf(wm, q.x, fmaf(w0, q.y, v.y));
                            }
                        }
                }
                // elements near the row's ends: edge samples replicated
#pragma unroll
                for (int b = 0; b < NB1; ++b)
#pragma unroll
                    for (int t = 0; t < H1; ++t) {
                        const int e = T + b * TN + t * (M / R1);
                        if (live && 2 * e < nc && !(e >= K && 2 * e + 1 + 2 * K < nc)) {
                            float v[2] = {0.0f, 0.0f};
                            for (int h = 0; h < 2; ++h) {
                                const int j = 2 * e + h;
                                if (j < nc)
                                    for (int m = -R; m <= R; ++m)
                                        v[h] = fmaf(pre.taps[m + R], stage[min(max(j + m, 0), nc - 1)], v[h]);
                            }
                            x[b * R1 + t] = make_float2(v[0], v[1]);
                        }
                    }
            }
            __syncthreads();  // the staged row is read before P1 overwrites it
        }

        // ---- P1 (span 1): outputs s of butterfly j at positions R1 j + s
        {
            const int sb = 8 * lpos(rb + R1 * T);
#pragma unroll
            for (int b = 0; b < NB1; ++b) {
                dft<R1, false>(x + b * R1);
#pragma unroll
                for (int s = 0; s < R1; ++s) lds_at(z, sb, b * R1 * TN + s) = x[b * R1 + dft_slot<R1>(s)];
            }
        }
        // spectrum factors of the last pass's positions A + s NS and
        // B + s NS, then the next group's samples: loads complete in order,
        // so the wait for these factors does not wait for the prefetch
        float HA[16], HB[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            HA[s] = a.H[A + s * NS];
            HB[s] = a.H[B + s * NS];
        }
        const float HM = a.H[M];
        if constexpr (FEP) {
            const int64_t gn = g + gridDim.x, rn = gn * ROWS + rho;
            if (gn < groups && rn < a.rows) load_raw_quads<TN>(rq, a, rn, T);
        } else if constexpr (PERSIST) {
            const int64_t gn = g + gridDim.x, rn = gn * ROWS + rho;
            if (gn < groups && rn < a.rows) load_p1<R1, NB1, TN, M, TP, LMODE>(xn, a, rn, T);
        }
        __syncthreads();

        // ---- P2 (span R1): butterfly j = T + b TN reads j + t M/R2, writes
        // (j - k) R2 + k + s R1 with k = j mod R1
        if constexpr (R2 > 1) {
            {
                const int sb = 8 * lpos(rb + T);
#pragma unroll
                for (int b = 0; b < NB2; ++b)
#pragma unroll
                    for (int t = 0; t < R2; ++t) x[b * R2 + t] = lds_at(z, sb, b * TN + t * (M / R2));
            }
            __syncthreads();
            float2 tw2[R2];
            if constexpr (R2 == 16) {
                powers16(w21, w24, tw2);
            } else {
                tw2[0] = make_float2(1.0f, 0.0f);
                tw2[1] = w21;
                tw2[2] = cmul(w21, w21);
                tw2[3] = cmul(tw2[2], w21);
            }
#pragma unroll
            for (int b = 0; b < NB2; ++b) {
#pragma unroll
                for (int t = 1; t < R2; ++t) x[b * R2 + t] = cmul(x[b * R2 + t], tw2[t]);
                dft<R2, false>(x + b * R2);
            }
            const int sb = 8 * lpos(rb + (T - k2) * R2 + k2);
#pragma unroll
            for (int b = 0; b < NB2; ++b)
#pragma unroll
                for (int s = 0; s < R2; ++s) lds_at(z, sb, b * TN * R2 + s * R1) = x[b * R2 + dft_slot<R2>(s)];
            __syncthreads();
        }

        // ---- P3 (span NS) on butterflies A and B, spectrum, P3^H
        float2 *xa = x, *xb = x + 16;
        {
            const int sbA = 8 * lpos(rb + A), sbB = 8 * lpos(rb + B);
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                xa[t] = lds_at(z, sbA, t * NS);
                xb[t] = lds_at(z, sbB, t * NS);
            }
        }
        // no barrier: P3^H writes back exactly the positions this thread read
        {
            float2 pA[16], pB[16];
            powers16(w1A, w4A, pA);
            powers16(w1B, w4B, pB);
#pragma unroll
            for (int t = 1; t < 16; ++t) {
                xa[t] = cmul(xa[t], pA[t]);
                xb[t] = cmul(xb[t], pB[t]);
            }
        }
        dft<16, false>(xa);
        dft<16, false>(xb);
        // Z at position A + s NS is xa[dft_slot<16>(s)]; Z' replaces it there.
#define XA(s) xa[dft_slot<16>(s)]
#define XB(s) xb[dft_slot<16>(s)]
        if (T == 0) {
            // butterfly 0: pairs (s NS, (16 - s) NS), with bins 0 and M/2
            // paired with themselves (H[M]: the real row's Nyquist bin);
            // butterfly NS/2: pairs (NS/2 + s NS, NS/2 + (15 - s) NS);
            // W^(s NS) = exp(-2 pi i s / 32)
            float2 d;
            spectrum_pair(XA(0), XA(0), make_float2(1.0f, 0.0f), HA[0], HM, XA(0), d);
            spectrum_pair(XA(8), XA(8), make_float2(0.0f, -1.0f), HA[8], HA[8], XA(8), d);
#pragma unroll
            for (int s = 1; s < 8; ++s)
                spectrum_pair(XA(s), XA(16 - s), root<false>(s, 32), HA[s], HA[16 - s], XA(s), XA(16 - s));
#pragma unroll
            for (int s = 0; s < 8; ++s)
                spectrum_pair(XB(s), XB(15 - s), root<false>(2 * s + 1, 64), HB[s], HB[15 - s], XB(s), XB(15 - s));
        }
        if (T != 0) {
            // pairs (A + s NS, M - A - s NS = B + (15 - s) NS), W^(T + s NS)
#pragma unroll
            for (int s = 0; s < 16; ++s)
                spectrum_pair(XA(s), XB(15 - s), turn<false>(WT, s, 32), HA[s], HB[15 - s], XA(s), XB(15 - s));
        }
        // P3^H: DFT^H over s (inputs in natural order), conj twiddles, to A + t NS
        {
            float2 ya[16], yb[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                ya[s] = XA(s);
                yb[s] = XB(s);
            }
#undef XA
#undef XB
            dft<16, true>(ya);
            dft<16, true>(yb);
            float2 pA[16], pB[16];
            powers16(opaque(w1A), opaque(w4A), pA);
            powers16(opaque(w1B), opaque(w4B), pB);
            const int sbA = opaque_i(8 * lpos(rb + A)), sbB = opaque_i(8 * lpos(rb + B));
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const float2 va = ya[dft_slot<16>(t)], vb = yb[dft_slot<16>(t)];
                lds_at(z, sbA, t * NS) = t ? cconj_mul(va, pA[t]) : va;
                lds_at(z, sbB, t * NS) = t ? cconj_mul(vb, pB[t]) : vb;
            }
        }
        __syncthreads();

        // ---- P2^H
        if constexpr (R2 > 1) {
            {
                const int sb = opaque_i(8 * lpos(rb + (T - k2) * R2 + k2));
#pragma unroll
                for (int b = 0; b < NB2; ++b)
#pragma unroll
                    for (int s = 0; s < R2; ++s) x[b * R2 + s] = lds_at(z, sb, b * TN * R2 + s * R1);
            }
            __syncthreads();
            float2 tw2[R2];
            if constexpr (R2 == 16) {
                powers16(opaque(w21), opaque(w24), tw2);
            } else {
                const float2 w = opaque(w21);
                tw2[0] = make_float2(1.0f, 0.0f);
                tw2[1] = w;
                tw2[2] = cmul(w, w);
                tw2[3] = cmul(tw2[2], w);
            }
            const int sb = opaque_i(8 * lpos(rb + T));
#pragma unroll
            for (int b = 0; b < NB2; ++b) {
                dft<R2, true>(x + b * R2);
#pragma unroll
                for (int t = 0; t < R2; ++t) {
                    const float2 v = x[b * R2 + dft_slot<R2>(t)];
                    lds_at(z, sb, b * TN + t * (M / R2)) = t ? cconj_mul(v, tw2[t]) : v;
                }
            }
            __syncthreads();
        }

        // ---- P1^H: DFT^H of the R1 values at positions R1 j + s, to elements
        // j + t M/R1 of the output row (element e = samples 2e, 2e + 1)
        {
            const int sb = opaque_i(8 * lpos(rb + R1 * T));
#pragma unroll
            for (int b = 0; b < NB1; ++b) {
#pragma unroll
                for (int s = 0; s < R1; ++s) x[b * R1 + s] = lds_at(z, sb, b * R1 * TN + s);
                dft<R1, true>(x + b * R1);
            }
        }
        // The next group's P1 writes the positions this thread's P1^H read
        // and nothing else; only the front end's staging of a raw row
        // touches other threads' positions.
        if constexpr (PRE) __syncthreads();
        if (live) {
            if (out_t == XCT_F32) store_p1<R1, NB1, TN, M, float>(x, a, r, T);
            else if (out_t == XCT_F16) store_p1<R1, NB1, TN, M, f16_t>(x, a, r, T);
            else store_p1<R1, NB1, TN, M, bf16_t>(x, a, r, T);
        }
    };
    if constexpr (PERSIST) {
        for (; g < groups; g += gridDim.x) group(g);
    } else {
        if (g < groups) group(g);
    }
}

template <typename TI, typename TO, bool PRE>
static hipError_t launch_typed(const FilterArgs &a, hipStream_t s)
{
    const int M = a.L >> 1;
    const int nt = max(64, min(1024, M / 16));  // M / nt <= 16 packed elements per thread
    // packed row + twiddles (the table rounded up to whole 32-entry groups,
    // which its swizzle permutes within)
    const size_t lds = (size_t)(M + ((M / 8 + 1 + 31) & ~31)) * sizeof(float2);
    (void)hipGetLastError();  // report only what this launch does
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(filter_small_kernel<TI, TO, PRE>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // one workgroup per row; a grid is at most 2^32 - 1 work-items
    const int64_t max_rows = ((((int64_t)1 << 32) - 1) / nt);
    FilterArgs c = a;
    for (int64_t r0 = 0; r0 < a.rows; r0 += max_rows) {
        c.row_base = r0;
        const int64_t n = a.rows - r0 < max_rows ? a.rows - r0 : max_rows;
        hipLaunchKernelGGL((filter_small_kernel<TI, TO, PRE>), dim3((unsigned)n), dim3(nt), lds, s, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TI, bool PRE>
static hipError_t launch_out(const FilterArgs &a, int out_t, hipStream_t s)
{
    if (out_t == XCT_F32) return launch_typed<TI, float, PRE>(a, s);
    if (out_t == XCT_F16) return launch_typed<TI, f16_t, PRE>(a, s);
    return launch_typed<TI, bf16_t, PRE>(a, s);
}

template <int KIND>
static hipError_t launch_kind(int lg, unsigned n, const FilterArgs &a, int in_t, int out_t, hipStream_t s)
{
    switch (lg) {
    case 8: hipLaunchKernelGGL((filter_fused_kernel<8, KIND>), dim3(n), dim3(256), 0, s, a, in_t, out_t); break;
    case 9: hipLaunchKernelGGL((filter_fused_kernel<9, KIND>), dim3(n), dim3(256), 0, s, a, in_t, out_t); break;
    case 10: hipLaunchKernelGGL((filter_fused_kernel<10, KIND>), dim3(n), dim3(256), 0, s, a, in_t, out_t); break;
    case 11: hipLaunchKernelGGL((filter_fused_kernel<11, KIND>), dim3(n), dim3(256), 0, s, a, in_t, out_t); break;
    case 12: hipLaunchKernelGGL((filter_fused_kernel<12, KIND>), dim3(n), dim3(256), 0, s, a, in_t, out_t); break;
    default: hipLaunchKernelGGL((filter_fused_kernel<13, KIND>), dim3(n), dim3(256), 0, s, a, in_t, out_t); break;
    }
    return hipGetLastError();
}

// Rows of 256 <= M <= 8192.  Unshifted, unweighted rows of even length in
// a buffer aligned to two samples, and front ends from uint16 counts over N_c
// a multiple of 4 with the stack aligned to 8 bytes and the fields to 16, take a
// persistent kernel: two workgroups per CU (as many as the LDS holds), each
// walking its groups of rows with the next group's samples in flight; so do
// FP32 rows of any other form (shifted, weighted, odd), loaded sample by
// sample.  Other rows take a workgroup per group (at most 2^32 - 1
// work-items: N_c <= 8192 keeps the groups of any valid call below that).
static hipError_t launch_fused(const FilterArgs &a, bool pre, int in_t, int out_t, hipStream_t s)
{
    const int lg = a.log2L - 1;  // log2 M
    const int rows_per_wg = 8192 >> lg;
    const int64_t wgs = (a.rows + rows_per_wg - 1) / rows_per_wg;
    const size_t esz = in_t == XCT_F32 ? 4 : 2;
    const bool plain = !a.weight && a.in_first == 0 && (a.in_len & 1) == 0 &&
                       reinterpret_cast<uintptr_t>(a.in) % (2 * esz) == 0;
    const bool persist = pre ? in_t == XCT_U16 && (a.nc & 3) == 0 && reinterpret_cast<uintptr_t>(a.in) % 8 == 0 &&
                                   reinterpret_cast<uintptr_t>(a.pre.dark) % 16 == 0 &&
                                   reinterpret_cast<uintptr_t>(a.pre.flat) % 16 == 0
                             : plain || in_t == XCT_F32;
    const int64_t cap = persist ? 2 * (int64_t)device_cus() : (((int64_t)1 << 32) - 1) / 256;
    if (!persist && wgs > cap) return hipErrorInvalidConfiguration;
    const unsigned n = (unsigned)(wgs < cap ? wgs : cap);
    (void)hipGetLastError();  // report only what this launch does
    if (pre && persist) return launch_kind<kPersistFE16>(lg, n, a, in_t, out_t, s);
    if (pre) return launch_kind<kFrontEnd>(lg, n, a, in_t, out_t, s);
    if (!persist) return launch_kind<kRows>(lg, n, a, in_t, out_t, s);
    if (!plain) return launch_kind<kPersistAnyF32>(lg, n, a, in_t, out_t, s);
    if (in_t == XCT_F32) return launch_kind<kPersistF32>(lg, n, a, in_t, out_t, s);
    if (in_t == XCT_F16) return launch_kind<kPersistF16>(lg, n, a, in_t, out_t, s);
    return launch_kind<kPersistBF16>(lg, n, a, in_t, out_t, s);
}

hipError_t launch_filter(const FilterArgs &a, int in_t, int out_t, hipStream_t s)
{
    if (a.log2L - 1 >= 8) return launch_fused(a, false, in_t, out_t, s);
    if (in_t == XCT_F32) return launch_out<float, false>(a, out_t, s);
    if (in_t == XCT_F16) return launch_out<f16_t, false>(a, out_t, s);
    return launch_out<bf16_t, false>(a, out_t, s);
}

hipError_t launch_front_end_filter(const FilterArgs &a, int in_t, int out_t, hipStream_t s)
{
    if (a.log2L - 1 >= 8) return launch_fused(a, true, in_t, out_t, s);
    if (in_t == XCT_U16) return launch_out<uint16_t, true>(a, out_t, s);
    return launch_out<float, true>(a, out_t, s);
}

}  // namespace xct
