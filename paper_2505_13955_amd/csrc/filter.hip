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
// One workgroup filters one row.  The real row x of length L = 2M is packed as
// z[n] = x[2n] + i x[2n+1] and transformed with one complex FFT of length M;
// a single pass over the bin pairs (k, M - k) recovers the real row's spectrum
//   X[k] = E + W^k O,  X[M-k] = conj(E - W^k O),  W = exp(-2 pi i / L),
//   E = (Z[k] + conj Z[M-k]) / 2,  O = (Z[k] - conj Z[M-k]) / 2i,
// multiplies it by H, and packs Y = H X back into Z'[k] = (Y[k] + conj
// Y[M-k]) + i (Y[k] - conj Y[M-k]) W^-k, whose inverse FFT of length M holds
// the filtered row as y[2n] + i y[2n+1].  The factors 1/2 and 1/M and the
// 1/pitch fold into H / (L pitch).  The inverse is done as the conjugate of
// the forward transform of conj Z'.
//
// The transform lives in LDS (M <= 8192 complex FP32 = 64 KiB, plus 8 KiB of
// twiddles, so two workgroups share a CU) and runs as mixed-radix Stockham passes (radix 4,
// plus one radix-2 pass when log2 M is odd); each pass reads its operands
// into registers, synchronises, and writes the results in place.  Twiddles
// come from a table of exp(-2 pi i e / L) computed on the host in FP64; the
// passes read an eighth-turn copy of it held in LDS (M/8 + 1 entries).
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
__device__ __forceinline__ float beer_lambert(float i, float d, float f, float floor)
{
    return -logf(fmaxf(i - d, floor) / fmaxf(f - d, floor));
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
__global__ __launch_bounds__(1024) void filter_kernel(FilterArgs a)
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
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(filter_kernel<TI, TO, PRE>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // one workgroup per row; a grid is at most 2^32 - 1 work-items
    const int64_t max_rows = ((((int64_t)1 << 32) - 1) / nt);
    FilterArgs c = a;
    for (int64_t r0 = 0; r0 < a.rows; r0 += max_rows) {
        c.row_base = r0;
        const int64_t n = a.rows - r0 < max_rows ? a.rows - r0 : max_rows;
        hipLaunchKernelGGL((filter_kernel<TI, TO, PRE>), dim3((unsigned)n), dim3(nt), lds, s, c);
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
