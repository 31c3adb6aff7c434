// Back-projection kernels for gfx950.
//
// Back-projection (Section IV-B, second step of FBP; cost O(N_p N_x N_y) per
// slice, Section V-A c) sums, for every pixel, the linearly interpolated value
// of every filtered projection row at the pixel's detector coordinate
//   u_k(x, y) = x C_k + y S_k + c,   C_k = cos(th_k) pix/pitch, S_k = sin(th_k) pix/pitch.
//
// Work decomposition.  A workgroup of 256 threads owns a 64 x 64 pixel tile
// and walks all angles in LDS stages.  For each angle of a stage the part of
// the row the tile can touch (a window of W ~ 63 sqrt(2) + 3 bins) is copied
// into LDS once, pre-paired so that the inner loop needs one 8-byte LDS read
// and one FMA per interpolation: entry m of a window that starts at bin B
// holds d = q[B+m+1] - q[B+m] and a = q[B+m] - m d, so that for the local
// coordinate u = (detector coordinate) - B, in [m, m+1),
//   q[B+m] (1 - t) + q[B+m+1] t  =  a + u d,   t = u - m,
// and the fraction t never has to be formed.  Each thread keeps
// 16 pixels (a 4 x 4 lattice with stride 16) in registers; a wavefront covers
// an 8 x 8 pixel block, whose detector footprint spans at most 12 bins, so its
// LDS reads hit distinct banks or broadcast.
//
// Precision.  Detector coordinates are formed relative to the window start,
// which the window-anchor step computes in FP64 per (tile, angle); the FP32
// value that reaches the inner loop is then below W and carries ~1e-5 bin of
// rounding even at 8192 bins.  Filtered rows stored as FP16 / BF16 are widened
// exactly while staging; interpolation and accumulation are FP32 throughout.
//
// Two kernels:
//  * bp_generic: any geometry (angles, centre, rectangular slices).
//  * bp_sym:     square slices of even size, angle sets closed under
//    th -> th + pi/2 (N_p even, th_{k+N_p/2} = th_k + pi/2) and 2c integral.
//    Then the detector coordinate of pixel Q at th_k also gives, through the
//    quarter-turn rotation R(x, y) = (y, -x) and the mirror u -> 2c - u of
//    the detector, the coordinates of R^2 Q at th_k and of R^3 Q and R Q at
//    th_k + pi/2.  One coordinate and one floor then serve four updates,
//    read from four windows that share one local coordinate.  The workgroup
//    owns a tile of the top-left quadrant and its three rotations; with two
//    slices per work item (512 threads) each thread keeps 8 pixels x 4
//    rotations x 2 slices, and one 16-byte LDS read (a bin's pair and its
//    mirror's) serves two updates.
#include <cstring>

#include "xct_internal.h"

namespace xct {

template <typename T>
__device__ __forceinline__ float load_elem(const T *p, int64_t i);
template <>
__device__ __forceinline__ float load_elem<float>(const float *p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float load_elem<f16_t>(const f16_t *p, int64_t i) { return (float)p[i]; }
template <>
__device__ __forceinline__ float load_elem<bf16_t>(const bf16_t *p, int64_t i)
{
    return __uint_as_float((uint32_t)p[i].bits << 16);
}

// Zero-extended row element: q[n] for n in [0, nc), else 0.
template <typename T>
__device__ __forceinline__ float row_elem(const T *row, int n, int nc)
{
    return (n >= 0 && n < nc) ? load_elem(row, n) : 0.0f;
}

// The batch descriptor is the kernel's only argument, so it sits at offset 0
// of the kernarg segment.  Reading it through a constant-address-space
// pointer to that segment keeps the dynamically indexed slab table in scalar
// loads: every field read from it is wave-uniform (an SGPR), as are the rows
// and buffer resources derived from it, and nothing is copied to scratch.  A
// launch over more slabs than the arguments hold reads the descriptors from
// a device table through the same (constant) address space, which also keeps
// them in scalar loads (the table is written by an earlier launch on the same
// stream, and every launch starts with the scalar cache invalidated).
typedef const __attribute__((address_space(4))) BPBatch KBatch;
typedef const __attribute__((address_space(4))) BPSlab KSlab;

__device__ __forceinline__ KBatch *kernarg_batch()
{
    return (KBatch *)__builtin_amdgcn_kernarg_segment_ptr();
}

__device__ __forceinline__ KSlab *slab_at(KBatch *b, int s)
{
    if (b->table) return (KSlab *)(uintptr_t)b->table + s;
    return &b->slab[s];
}

__device__ __forceinline__ void select_slab(KBatch *b, int s, BPSlab &out)
{
    KSlab *d = slab_at(b, s);
    out.sino = d->sino;
    out.image = d->image;
    out.cs = d->cs;
    out.csd = d->csd;
    out.center = d->center;
    out.item_begin = d->item_begin;
    out.n_angles = d->n_angles;
    out.n_det = d->n_det;
    out.nx = d->nx;
    out.ny = d->ny;
    out.n_slices = d->n_slices;
    out.tiles_x = d->tiles_x;
    out.tiles_y = d->tiles_y;
    out.mirror = d->mirror;
    out.scale = d->scale;
    out.accumulate = d->accumulate;
    out.out_u16 = d->out_u16;
    out.code_a = d->code_a;
    out.code_b = d->code_b;
    out.sets = d->sets;
}

// Store of voxel `idx` (slab-wide index) from its accumulated sum: v = scale
// * acc in FP32 (added to the stored value when accumulating), or the CT-number
// code of v: the affine map fl(fl(v a) + b) rounded to the nearest integer,
// ties to even, and clamped to [0, 65535] (NaN gives 0).  The explicit
// roundings keep the code independent of FMA contraction.
__device__ __forceinline__ void store_voxel(const BPSlab &sl, int64_t idx, float acc)
{
    float v = sl.scale * acc;
    if (sl.out_u16) {
        const float t = __fadd_rn(__fmul_rn(v, sl.code_a), sl.code_b);
        const float c = fminf(fmaxf(rintf(t), 0.0f), 65535.0f);
        static_cast<uint16_t *>(sl.image)[idx] = (uint16_t)c;
    } else {
        float *img = static_cast<float *>(sl.image);
        if (sl.accumulate) v += img[idx];
        img[idx] = v;
    }
}

// Slab of a work item: the last slab whose first item is at or before it
// (binary search over the increasing item_begin; uniform, scalar loads).
__device__ __forceinline__ int find_slab(KBatch *b, int64_t item)
{
    int lo = 0, hi = b->n_slabs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (slab_at(b, mid)->item_begin <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The same value in every lane, as a scalar: everything derived from it
// (slab, rows, buffer resources) then stays wave-uniform.
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v) |
           ((int64_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32);
}

// Next work item of this workgroup; a value >= total_items when it is done.
//  * Non-persistent launch: one item per workgroup, item_base + the block
//    index, optionally remapped so that XCD x (blocks x, x + 8, ...) takes the
//    contiguous range [x n/8, (x+1) n/8) of the launch's n items.
//  * Persistent launch: the items are dealt to the XCDs in bundles of
//    kXcdBundle consecutive items (bundle i to XCD i mod 8), and each XCD
//    walks its own bundles in order with its own counter, so the global order
//    (most expensive slab first) is kept while one XCD's workgroups take
//    neighbouring tiles.  A workgroup whose XCD has run out takes items from
//    the other XCDs' counters in turn.  Which XCD a workgroup runs on only
//    affects locality: every item is taken exactly once either way.
__device__ __forceinline__ int64_t next_item(KBatch *b, int64_t *slot, int iter)
{
    if (b->counter) {
        if (threadIdx.x == 0) {
            const int home = blockIdx.x % kXcds;
            int64_t it = b->total_items;
            for (int t = 0; t < kXcds; ++t) {
                const int x = (home + t) % kXcds;
                const unsigned c = atomicAdd(b->counter + x, 1u);
                const int64_t bundle = (int64_t)(c / kXcdBundle) * kXcds + x;
                const int64_t cand = bundle * kXcdBundle + c % kXcdBundle;
                if (cand < b->total_items) {
                    it = cand;
                    break;
                }
            }
            *slot = it;
        }
        __syncthreads();
        const int64_t it = *slot;
        __syncthreads();
        return it;
    }
    if (iter > 0) return b->total_items;
    int64_t bid = blockIdx.x;
    if (b->xcd_remap) {
        const int64_t per = gridDim.x >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    return b->item_base + bid;
}

// Pixel lattice of one thread inside a 64 x 64 tile: a wave covers an 8 x 8
// block, the four waves a 16 x 16 block, and the lattice repeats with stride 16.
__device__ __forceinline__ void thread_lattice(int tid, int &px, int &py)
{
    px = (tid & 7) | (((tid >> 6) & 1) << 3);
    py = ((tid >> 3) & 7) | ((tid >> 7) << 3);
}

// ---------------------------------------------------------------- generic

size_t bp_generic_lds_bytes(int win, int kb)
{
    return (size_t)kb * sizeof(float4) + (size_t)kb * win * sizeof(float2);
}

template <typename T>
__global__ __launch_bounds__(kBPThreads) void bp_generic_kernel(BPBatch arg)
{
    KBatch *b = kernarg_batch();
    extern __shared__ float4 lds4[];
    __shared__ int64_t item_slot;
    const int kb = b->kb, W = b->win;
    float4 *par = lds4;                          // (frac anchor, C, S, window start)
    float2 *win = reinterpret_cast<float2 *>(lds4 + kb);
    const int tid = threadIdx.x;
    int px, py;
    thread_lattice(tid, px, py);
    const float dxo = px - 31.5f, dyo = py - 31.5f;

    for (int iter = 0;; ++iter) {
        const int64_t item = uniform64(next_item(b, &item_slot, iter));
        if (item >= b->total_items) break;
        BPSlab sl;
        select_slab(b, find_slab(b, item), sl);
        const int64_t local = item - sl.item_begin;
        const int tiles = sl.tiles_x * sl.tiles_y;
        const int z = __builtin_amdgcn_readfirstlane((int)(local / tiles));
        const int t = __builtin_amdgcn_readfirstlane((int)(local - (int64_t)z * tiles));
        const int ty = t / sl.tiles_x, tx = t - ty * sl.tiles_x;
        const int i0 = ty * kTile, j0 = tx * kTile;
        const double xc = j0 + 31.5 - 0.5 * (sl.nx - 1);
        const double yc = i0 + 31.5 - 0.5 * (sl.ny - 1);
        const int Np = sl.n_angles, Nc = sl.n_det;
        const T *q = static_cast<const T *>(sl.sino) + (int64_t)z * Np * Nc;

        float acc[16];
#pragma unroll
        for (int p = 0; p < 16; ++p) acc[p] = 0.0f;

        for (int k0 = 0; k0 < Np; k0 += kb) {
            const int nk = min(kb, Np - k0);
            __syncthreads();
            if (tid < nk) {
                const double2 cd = sl.csd[k0 + tid];
                const double U = xc * cd.x + yc * cd.y + sl.center;
                const double E = 31.5 * (fabs(cd.x) + fabs(cd.y));
                const double B = floor(U - E) - 1.0;
                const float2 cf = sl.cs[k0 + tid];
                par[tid] = make_float4((float)(U - B), cf.x, cf.y, __int_as_float((int)B));
            }
            __syncthreads();
            for (int e = tid; e < nk * W; e += kBPThreads) {
                const int kk = e / W, m = e - kk * W;
                const int n = __float_as_int(par[kk].w) + m;
                const T *row = q + (int64_t)(k0 + kk) * Nc;
                const float a0 = row_elem(row, n, Nc);
                const float d = row_elem(row, n + 1, Nc) - a0;
                win[e] = make_float2(fmaf(-(float)m, d, a0), d);
            }
            __syncthreads();
            for (int kk = 0; kk < nk; ++kk) {
                const float4 p = par[kk];
                const float2 *w = win + kk * W;
                const float c16 = 16.0f * p.y, s16 = 16.0f * p.z;
                float ur = p.x + dxo * p.y + dyo * p.z;
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    float u = ur;
#pragma unroll
                    for (int aa = 0; aa < 4; ++aa) {
                        const float2 v = w[(int)u];
                        acc[bb * 4 + aa] += fmaf(u, v.y, v.x);
                        u += c16;
                    }
                    ur += s16;
                }
            }
        }

        const int64_t plane = (int64_t)z * sl.nx * sl.ny;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
#pragma unroll
            for (int aa = 0; aa < 4; ++aa) {
                const int i = i0 + py + 16 * bb, j = j0 + px + 16 * aa;
                if (i < sl.ny && j < sl.nx) store_voxel(sl, plane + (int64_t)i * sl.nx + j, acc[bb * 4 + aa]);
            }
        }
    }
}

// ---------------------------------------------------------------- symmetric

// LDS stage of the symmetric kernel: per angle pair kk, the parameters
// (fbA, fbB, C, S) and window starts (B_A, B_B), then the windows.  Group A is
// anchored on u(Q, th_k), group B on u(R Q, th_k); each group has four
// windows: forward row k, mirrored row k, forward row k+H, mirrored row k+H,
// all indexed by the same local coordinate.  Structure of arrays, W entries
// of 16 bytes per array:
//   [A: row k (a,d) fwd + (a,d) mirrored][A: row k+H][B: row k][B: row k+H]
// so the 16-byte reads of a wavefront land on consecutive 16-byte slots (no
// bank conflicts while its footprint spans fewer than 16 entries).
size_t bp_sym_lds_bytes(int win, int kb, int sl)
{
    const size_t head = ((size_t)kb + ((size_t)kb + 1) / 2) * sizeof(float4);
    return head + (size_t)kb * 4 * win * sl * sizeof(float4);
}

// Buffer resource over one sinogram row: the buffer unit's range check
// returns 0 for byte offsets at or past the row's end, which gives the zero
// extension on the far side of the detector without a compare.  Offsets
// below the row start are redirected (kBeyond) to the same range check.
constexpr uint32_t kBeyond = 0x40000000u;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T *row, int nc)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(row), (short)0, nc * (int)sizeof(T),
                                             0x00020000);
}

// Byte offset of element n of a row (kBeyond for n < 0).
template <typename T>
__device__ __forceinline__ uint32_t elem_offset(int n)
{
    return n >= 0 ? (uint32_t)n * (uint32_t)sizeof(T) : kBeyond;
}

template <typename T>
__device__ __forceinline__ float buf_elem(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float buf_elem<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_elem<f16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return (float)__builtin_bit_cast(f16_t, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_elem<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0) << 16);
}

// Tile of work item t within a slice (group): row-major, or, with
// XCT_TILE_GROUP = G > 1 and both tile counts divisible by G, row-major over
// G x G groups of tiles so that consecutive items (which run together on one
// XCD) cover a compact region and share more detector windows in L2.
#ifndef XCT_TILE_GROUP
#define XCT_TILE_GROUP 4
#endif
__device__ __forceinline__ void tile_position(int t, int tiles_x, int tiles_y, int &ty, int &tx)
{
    constexpr int G = XCT_TILE_GROUP;
    if (G > 1 && tiles_x % G == 0 && tiles_y % G == 0) {
        const int grp = t / (G * G), in = t - grp * (G * G);
        const int gy = grp / (tiles_x / G), gx = grp - gy * (tiles_x / G);
        ty = gy * G + in / G;
        tx = gx * G + in % G;
    } else {
        ty = t / tiles_x;
        tx = t - ty * tiles_x;
    }
}

#ifndef XCT_STAGE_UNITS
#define XCT_STAGE_UNITS 5  // staging units whose loads are in flight together
#endif

// SL slices per work item: every slice of a slab shares the geometry, so the
// coordinates, floors and LDS addresses of one tile serve all SL slices; only
// the windows differ.  With SL = 2 the workgroup has 512 threads and each
// keeps 8 pixels x 4 rotations x 2 slices in registers.
template <int SL>
constexpr int sym_threads() { return SL == 2 ? XCT_SYM2_THREADS : kBPThreads; }
template <int SL>
constexpr int sym_waves() { return SL == 2 ? XCT_SYM2_WAVES : 4; }

template <typename T, int W, int SL>
__global__ __launch_bounds__(sym_threads<SL>(), sym_waves<SL>()) void bp_sym_kernel(BPBatch arg)
{
    KBatch *b = kernarg_batch();
    extern __shared__ float4 lds4[];
    __shared__ int64_t item_slot;
    constexpr int kThreads = sym_threads<SL>();
    constexpr int PX = 4096 / kThreads;  // pixels per thread
    constexpr int ROWS = PX / 4;         // lattice rows per thread
    constexpr int RS = kThreads / 16;    // lattice row stride
    constexpr int PER = 4 * W * SL;      // float4 per angle pair
    const int kb = b->kb;
    float4 *par = lds4;
    int2 *wstart = reinterpret_cast<int2 *>(lds4 + kb);
    float4 *win = lds4 + kb + (kb + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // a wave covers an 8 x 8 block, the waves a 16 x RS block; each thread
    // has pixels (px + 16 a, py + RS c), a < 4, c < ROWS
    const int px = (lane & 7) | ((wv & 1) << 3);
    const int py = (lane >> 3) | ((wv >> 1) << 3);
    const float dxo = px - 31.5f, dyo = py - 31.5f;

    for (int iter = 0;; ++iter) {
        const int64_t item = uniform64(next_item(b, &item_slot, iter));
        if (item >= b->total_items) break;
        BPSlab sl;
        select_slab(b, find_slab(b, item), sl);
        const int64_t local = item - sl.item_begin;
        const int tiles = sl.tiles_x * sl.tiles_y;
        // slice group and tile (the 64-bit division runs on the vector unit;
        // pin the results back to scalars)
        const int zg = __builtin_amdgcn_readfirstlane((int)(local / tiles));
        const int t = __builtin_amdgcn_readfirstlane((int)(local - (int64_t)zg * tiles));
        int ty, tx;
        tile_position(t, sl.tiles_x, sl.tiles_y, ty, tx);
        const int N = sl.nx, half = N >> 1;
        const int i0 = ty * kTile, j0 = tx * kTile;
        const double xc = j0 + 31.5 - 0.5 * (N - 1);
        const double yc = i0 + 31.5 - 0.5 * (N - 1);
        // the angle set is `sets` consecutive half-turn sets (a full turn is
        // two); in each, angle k + H is angle k plus a quarter turn
        const int Np = sl.n_angles, Nc = sl.n_det, H = (Np / sl.sets) >> 1, M = sl.mirror;
        const int z0 = zg * SL;
        const int nsl = min(SL, sl.n_slices - z0);  // slices present in this group
        // first slice of the group, pinned to a scalar so the row buffer
        // resources built from it are wave-uniform
        const T *q = reinterpret_cast<const T *>(
            uniform64(reinterpret_cast<int64_t>(static_cast<const T *>(sl.sino) + (int64_t)z0 * Np * Nc)));
        const int64_t sl_stride = (int64_t)Np * Nc;  // elements between slices
        const int64_t h_stride = (int64_t)H * Nc;    // from row k to row k + H

        float acc[SL][4][PX];
#pragma unroll
        for (int s = 0; s < SL; ++s)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int p = 0; p < PX; ++p) acc[s][r][p] = 0.0f;

        // stages of up to kb angle pairs k0 .. k0+nk-1 (with k0+H ..); kc
        // counts pairs over the sets, and a stage never crosses a set
        for (int kc = 0, nk = 0; kc < sl.sets * H; kc += nk) {
            const int set = kc / H;
            const int k0 = kc + set * H;
            nk = min(kb, (set + 1) * H - kc);
            __syncthreads();
            if (tid < nk) {
                const double2 cd = sl.csd[k0 + tid];
                const double E = 31.5 * (fabs(cd.x) + fabs(cd.y));
                const double UA = xc * cd.x + yc * cd.y + sl.center;   // Q at th_k
                const double UB = yc * cd.x - xc * cd.y + sl.center;   // R Q at th_k
                const double BA = floor(UA - E) - 1.0, BB = floor(UB - E) - 1.0;
                const float2 cf = sl.cs[k0 + tid];
                par[tid] = make_float4((float)(UA - BA), (float)(UB - BB), cf.x, cf.y);
                wstart[tid] = make_int2((int)BA, (int)BB);
            }
            __syncthreads();
            // Each wavefront stages 64 entries of one angle pair of one slice
            // at a time (a unit), so the two rows are wave-uniform buffer
            // resources; a slice missing from the last group stages zeros
            // (empty resource).  The loads of XCT_STAGE_UNITS units are all
            // issued before the first is used, so a stage waits for one global
            // latency per group of units rather than one per unit; a unit
            // past the end loads through an empty resource and stores nothing.
            constexpr int kParts = 2 * W / 64;
            constexpr int kU = XCT_STAGE_UNITS;
            constexpr int kWaves = kThreads / 64;
            constexpr int D = SL * kParts;  // units per angle pair
            const int wave = __builtin_amdgcn_readfirstlane(wv);
            const int nunits = nk * D;
            // Unit u of the stage is angle pair u / D, slice (u % D) / kParts,
            // part (u % D) % kParts.  A wavefront's units are kWaves apart, so
            // the pair and remainder advance by scalar adds, and the rows are
            // addressed from the stage's first row: few scalar instructions
            // per unit.
            auto advance = [](int &kk, int &rest, int units) {
                kk += units / D;
                rest += units % D;
                if (rest >= D) {
                    rest -= D;
                    ++kk;
                }
            };
            const T *qk = q + (int64_t)k0 * Nc;  // row k0 of the group's first slice
            int kk0 = wave / D, rest0 = wave % D;
            for (int u0 = wave; u0 < nunits; u0 += kU * kWaves) {
                float v[kU][8];
                int kk = kk0, rest = rest0;
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    // (the buffer resource inputs pinned to scalars, so the
                    // loads need no waterfall loops)
                    const bool live = u0 + u * kWaves < nunits;
                    const int kl = __builtin_amdgcn_readfirstlane(live ? kk : 0);  // dead units: pair 0, empty resource
                    const int sidx = SL == 1 ? 0 : __builtin_amdgcn_readfirstlane(rest >= kParts);
                    const int e = (rest - sidx * kParts) * 64 + lane;  // entry of the pair, [0, 2W)
                    const int g = e >= W, m = e - g * W;
                    const int2 ws = wstart[kl];
                    const int n = (g ? ws.y : ws.x) + m;
                    const int rn = M - n;
                    const T *row = reinterpret_cast<const T *>(uniform64(
                        reinterpret_cast<int64_t>(qk + (sidx ? sl_stride : (int64_t)0) + kl * Nc)));
                    const int len = __builtin_amdgcn_readfirstlane((live && sidx < nsl) ? Nc : 0);
                    const auto rk = row_rsrc(row, len);
                    const auto rh = row_rsrc(row + h_stride, len);
                    const uint32_t o0 = elem_offset<T>(n), o1 = elem_offset<T>(n + 1);
                    const uint32_t r0 = elem_offset<T>(rn), r1 = elem_offset<T>(rn - 1);
                    v[u][0] = buf_elem<T>(rk, o0);
                    v[u][1] = buf_elem<T>(rk, o1);
                    v[u][2] = buf_elem<T>(rk, r0);
                    v[u][3] = buf_elem<T>(rk, r1);
                    v[u][4] = buf_elem<T>(rh, o0);
                    v[u][5] = buf_elem<T>(rh, o1);
                    v[u][6] = buf_elem<T>(rh, r0);
                    v[u][7] = buf_elem<T>(rh, r1);
                    advance(kk, rest, kWaves);
                }
                // keep the scheduler from sinking the loads back to their uses
                __builtin_amdgcn_sched_barrier(0);
                kk = kk0;
                rest = rest0;
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    if (u0 + u * kWaves >= nunits) break;
                    const int sidx = SL == 1 ? 0 : (rest >= kParts);
                    const int e = (rest - sidx * kParts) * 64 + lane;
                    const int g = e >= W, m = e - g * W;
                    const float f0 = v[u][0], fd = v[u][1] - f0, m0 = v[u][2], md = v[u][3] - m0;
                    const float h0 = v[u][4], hd = v[u][5] - h0, g0 = v[u][6], gd = v[u][7] - g0;
                    const float mf = -(float)m;
                    float4 *dst = win + kk * PER + sidx * 4 * W + g * 2 * W + m;
                    dst[0] = make_float4(fmaf(mf, fd, f0), fd, fmaf(mf, md, m0), md);
                    dst[W] = make_float4(fmaf(mf, hd, h0), hd, fmaf(mf, gd, g0), gd);
                    advance(kk, rest, kWaves);
                }
                advance(kk0, rest0, kU * kWaves);
            }
            __syncthreads();
            for (int kk = 0; kk < nk; ++kk) {
                const float4 p = par[kk];
                const float C = p.z, S = p.w;
                const float4 *wk = win + kk * PER;
                const float c16 = 16.0f * C, s16 = 16.0f * S;
                const float cr = (float)RS * C, sr = (float)RS * S;
                float ua_r = p.x + dxo * C + dyo * S;   // u(Q, th_k) - B_A
                float ub_r = p.y + dyo * C - dxo * S;   // u(R Q, th_k) - B_B
#pragma unroll
                for (int cc = 0; cc < ROWS; ++cc) {
                    float ua = ua_r, ub = ub_r;
#pragma unroll
                    for (int aa = 0; aa < 4; ++aa) {
                        const int na = (int)ua, nb = (int)ub;
                        const int pi = cc * 4 + aa;
#pragma unroll
                        for (int s = 0; s < SL; ++s) {
                            const float4 *ws = wk + s * 4 * W;
                            const float4 a0 = ws[na], a1 = ws[W + na];
                            const float4 b0 = ws[2 * W + nb], b1 = ws[3 * W + nb];
                            acc[s][0][pi] += fmaf(ua, a0.y, a0.x) + fmaf(ub, b1.y, b1.x);  // Q
                            acc[s][2][pi] += fmaf(ua, a0.w, a0.z) + fmaf(ub, b1.w, b1.z);  // R^2 Q
                            acc[s][3][pi] += fmaf(ua, a1.y, a1.x) + fmaf(ub, b0.w, b0.z);  // R^3 Q
                            acc[s][1][pi] += fmaf(ua, a1.w, a1.z) + fmaf(ub, b0.y, b0.x);  // R Q
                        }
                        ua += c16;
                        ub -= s16;
                    }
                    ua_r += sr;
                    ub_r += cr;
                }
            }
        }

#pragma unroll
        for (int s = 0; s < SL; ++s) {
            if (s >= nsl) break;
            const int64_t plane = (int64_t)(z0 + s) * N * N;
#pragma unroll
            for (int cc = 0; cc < ROWS; ++cc) {
#pragma unroll
                for (int aa = 0; aa < 4; ++aa) {
                    const int i = i0 + py + RS * cc, j = j0 + px + 16 * aa;
                    if (i < half && j < half) {
                        const int pi = cc * 4 + aa;
                        // Q = (i, j); R Q = (N-1-j, i); R^2 Q = (N-1-i, N-1-j); R^3 Q = (j, N-1-i)
                        const int64_t idx[4] = {(int64_t)i * N + j, (int64_t)(N - 1 - j) * N + i,
                                                (int64_t)(N - 1 - i) * N + (N - 1 - j),
                                                (int64_t)j * N + (N - 1 - i)};
#pragma unroll
                        for (int r = 0; r < 4; ++r) store_voxel(sl, plane + idx[r], acc[s][r][pi]);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- mirror

// Point reflection through the slice centre: pixel Q = (i, j) and
// R^2 Q = (N_y-1-i, N_x-1-j) have detector coordinates u and 2c - u at every
// angle (the pixel grid is centred), so with 2c integral one coordinate and
// one floor serve both, for any angle set and any slice shape.  A work item is
// a 64 x 64 tile of the upper half of the slice (rows below ceil(N_y/2)) and
// its reflection, all angles, SL slices.  Per angle the stage holds, for each
// slice, one window of W 16-byte entries (a, d) forward and (a, d) mirrored,
// indexed by the tile's local coordinate: one ds_read_b128 serves two
// updates.  Middle-row pixels of an odd N_y reflect into the same row, where
// they are their own tile's pixels: only Q is stored for them.
size_t bp_mirror_lds_bytes(int win, int kb, int sl)
{
    return (size_t)kb * sizeof(float4) + (size_t)kb * win * sl * sizeof(float4);
}

template <typename T, int W, int SL>
__global__ __launch_bounds__(sym_threads<SL>(), sym_waves<SL>()) void bp_mirror_kernel(BPBatch arg)
{
    KBatch *b = kernarg_batch();
    extern __shared__ float4 lds4[];
    __shared__ int64_t item_slot;
    constexpr int kThreads = sym_threads<SL>();
    constexpr int PX = 4096 / kThreads;  // pixels per thread
    constexpr int ROWS = PX / 4;         // lattice rows per thread
    constexpr int RS = kThreads / 16;    // lattice row stride
    constexpr int PER = W * SL;          // float4 per angle
    const int kb = b->kb;
    float4 *par = lds4;                  // (u(tile centre) - B, C, S, B as int bits)
    float4 *win = lds4 + kb;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int px = (lane & 7) | ((wv & 1) << 3);
    const int py = (lane >> 3) | ((wv >> 1) << 3);
    const float dxo = px - 31.5f, dyo = py - 31.5f;

    for (int iter = 0;; ++iter) {
        const int64_t item = uniform64(next_item(b, &item_slot, iter));
        if (item >= b->total_items) break;
        BPSlab sl;
        select_slab(b, find_slab(b, item), sl);
        const int64_t local = item - sl.item_begin;
        const int tiles = sl.tiles_x * sl.tiles_y;
        const int zg = __builtin_amdgcn_readfirstlane((int)(local / tiles));
        const int t = __builtin_amdgcn_readfirstlane((int)(local - (int64_t)zg * tiles));
        int ty, tx;
        tile_position(t, sl.tiles_x, sl.tiles_y, ty, tx);
        const int NX = sl.nx, NY = sl.ny, HY = (NY + 1) >> 1;
        const int i0 = ty * kTile, j0 = tx * kTile;
        const double xc = j0 + 31.5 - 0.5 * (NX - 1);
        const double yc = i0 + 31.5 - 0.5 * (NY - 1);
        const int Np = sl.n_angles, Nc = sl.n_det, M = sl.mirror;
        const int z0 = zg * SL;
        const int nsl = min(SL, sl.n_slices - z0);
        const T *q = reinterpret_cast<const T *>(
            uniform64(reinterpret_cast<int64_t>(static_cast<const T *>(sl.sino) + (int64_t)z0 * Np * Nc)));
        const int64_t sl_stride = (int64_t)Np * Nc;

        float acc[SL][2][PX];
#pragma unroll
        for (int s = 0; s < SL; ++s)
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int p = 0; p < PX; ++p) acc[s][r][p] = 0.0f;

        for (int k0 = 0, nk = 0; k0 < Np; k0 += nk) {
            nk = min(kb, Np - k0);
            __syncthreads();
            if (tid < nk) {
                const double2 cd = sl.csd[k0 + tid];
                const double E = 31.5 * (fabs(cd.x) + fabs(cd.y));
                const double U = xc * cd.x + yc * cd.y + sl.center;
                const double B = floor(U - E) - 1.0;
                const float2 cf = sl.cs[k0 + tid];
                par[tid] = make_float4((float)(U - B), cf.x, cf.y, __int_as_float((int)B));
            }
            __syncthreads();
            // Staging units of 64 entries: (angle, slice, part), the angle's
            // row a wave-uniform buffer resource (zero past the row's end,
            // negative bins redirected there), loads of kU units in flight.
            constexpr int kParts = (W + 63) / 64;
            constexpr int kU = XCT_STAGE_UNITS;
            constexpr int kWaves = kThreads / 64;
            constexpr int D = SL * kParts;  // units per angle
            const int wave = __builtin_amdgcn_readfirstlane(wv);
            const int nunits = nk * D;
            const T *qk = q + (int64_t)k0 * Nc;
            for (int u0 = wave; u0 < nunits; u0 += kU * kWaves) {
                float v[kU][4];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int unit = u0 + u * kWaves;
                    const bool live = unit < nunits;
                    const int kk = __builtin_amdgcn_readfirstlane(live ? unit / D : 0);
                    const int rest = __builtin_amdgcn_readfirstlane(live ? unit - kk * D : 0);
                    const int sidx = SL == 1 ? 0 : __builtin_amdgcn_readfirstlane(rest >= kParts);
                    const int m = (rest - sidx * kParts) * 64 + lane;
                    const int n = __float_as_int(par[kk].w) + m;
                    const int rn = M - n;
                    const T *row = reinterpret_cast<const T *>(uniform64(
                        reinterpret_cast<int64_t>(qk + (sidx ? sl_stride : (int64_t)0) + (int64_t)kk * Nc)));
                    const int len = __builtin_amdgcn_readfirstlane((live && sidx < nsl) ? Nc : 0);
                    const auto rk = row_rsrc(row, len);
                    v[u][0] = buf_elem<T>(rk, elem_offset<T>(n));
                    v[u][1] = buf_elem<T>(rk, elem_offset<T>(n + 1));
                    v[u][2] = buf_elem<T>(rk, elem_offset<T>(rn));
                    v[u][3] = buf_elem<T>(rk, elem_offset<T>(rn - 1));
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int unit = u0 + u * kWaves;
                    if (unit >= nunits) break;
                    const int kk = unit / D, rest = unit - kk * D;
                    const int sidx = SL == 1 ? 0 : (rest >= kParts);
                    const int m = (rest - sidx * kParts) * 64 + lane;
                    if (m < W) {
                        const float f0 = v[u][0], fd = v[u][1] - f0, m0 = v[u][2], md = v[u][3] - m0;
                        const float mf = -(float)m;
                        win[kk * PER + sidx * W + m] = make_float4(fmaf(mf, fd, f0), fd, fmaf(mf, md, m0), md);
                    }
                }
            }
            __syncthreads();
            for (int kk = 0; kk < nk; ++kk) {
                const float4 p = par[kk];
                const float C = p.y, S = p.z;
                const float4 *wk = win + kk * PER;
                const float c16 = 16.0f * C, sr = (float)RS * S;
                float u_r = p.x + dxo * C + dyo * S;  // u(Q) - B
#pragma unroll
                for (int cc = 0; cc < ROWS; ++cc) {
                    float u = u_r;
#pragma unroll
                    for (int aa = 0; aa < 4; ++aa) {
                        const int n = (int)u;
                        const int pi = cc * 4 + aa;
#pragma unroll
                        for (int s = 0; s < SL; ++s) {
                            const float4 a = wk[s * W + n];
                            acc[s][0][pi] += fmaf(u, a.y, a.x);   // Q
                            acc[s][1][pi] += fmaf(u, a.w, a.z);   // R^2 Q
                        }
                        u += c16;
                    }
                    u_r += sr;
                }
            }
        }

#pragma unroll
        for (int s = 0; s < SL; ++s) {
            if (s >= nsl) break;
            const int64_t plane = (int64_t)(z0 + s) * NX * NY;
#pragma unroll
            for (int cc = 0; cc < ROWS; ++cc) {
#pragma unroll
                for (int aa = 0; aa < 4; ++aa) {
                    const int i = i0 + py + RS * cc, j = j0 + px + 16 * aa;
                    if (i < HY && j < NX) {
                        const int pi = cc * 4 + aa;
                        store_voxel(sl, plane + (int64_t)i * NX + j, acc[s][0][pi]);
                        if (2 * i + 1 < NY)
                            store_voxel(sl, plane + (int64_t)(NY - 1 - i) * NX + (NX - 1 - j), acc[s][1][pi]);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- slab table

// Slab descriptors passed by value; the kernel copies them word by word from
// its argument segment into the device table with vector stores.
struct SlabChunk {
    BPSlab s[kInlineSlabs];
};
static_assert(sizeof(BPSlab) % 4 == 0, "slab descriptors are copied as 32-bit words");

__global__ __launch_bounds__(256) void write_slab_table_kernel(SlabChunk c, int n, BPSlab *dst)
{
    typedef const __attribute__((address_space(4))) uint32_t KWord;
    KWord *src = (KWord *)__builtin_amdgcn_kernarg_segment_ptr();  // c sits at offset 0
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    const int words = n * (int)(sizeof(BPSlab) / 4);
    for (int i = threadIdx.x; i < words; i += blockDim.x) d[i] = src[i];
}

hipError_t write_slab_table(BPSlab *dst, const BPSlab *src, int n, hipStream_t s)
{
    (void)hipGetLastError();
    for (int i = 0; i < n; i += kInlineSlabs) {
        const int m = n - i < kInlineSlabs ? n - i : kInlineSlabs;
        SlabChunk c;
        std::memset(&c, 0, sizeof(c));
        std::memcpy(c.s, src + i, sizeof(BPSlab) * (size_t)m);
        hipLaunchKernelGGL(write_slab_table_kernel, dim3(1), dim3(256), 0, s, c, m, dst + i);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- launchers

// Opt in to more than 64 KiB of dynamic LDS only when a launch needs it.
template <typename K>
static hipError_t prepare(K kernel, size_t lds)
{
    (void)hipGetLastError();  // report only what this launch does
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename K>
static hipError_t launch(K kernel, int threads, const BPBatch &b, int grid, size_t lds, hipStream_t s)
{
    hipError_t e = prepare(kernel, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, s, b);
    return hipGetLastError();
}

template <typename K>
static int occupancy(K kernel, int threads, size_t lds)
{
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, lds);
    (void)hipGetLastError();
    return (e == hipSuccess && n > 0) ? n : 1;
}

int bp_sym_window(int need) { return need <= 96 ? 96 : (need <= 192 ? 192 : 0); }

// The kernel instantiation for (path, filtered dtype, window, slices per
// item) and an action on it (launch or occupancy query), given the kernel
// and its block size.
template <int SL, typename F>
static auto with_sym(int dtype, int win, F &&f)
{
    constexpr int th = sym_threads<SL>();
    if (win == 96) {
        if (dtype == XCT_F32) return f(bp_sym_kernel<float, 96, SL>, th);
        if (dtype == XCT_F16) return f(bp_sym_kernel<f16_t, 96, SL>, th);
        return f(bp_sym_kernel<bf16_t, 96, SL>, th);
    }
    if (dtype == XCT_F32) return f(bp_sym_kernel<float, 192, SL>, th);
    if (dtype == XCT_F16) return f(bp_sym_kernel<f16_t, 192, SL>, th);
    return f(bp_sym_kernel<bf16_t, 192, SL>, th);
}

template <int SL, typename F>
static auto with_mirror(int dtype, int win, F &&f)
{
    constexpr int th = sym_threads<SL>();
    if (win == 96) {
        if (dtype == XCT_F32) return f(bp_mirror_kernel<float, 96, SL>, th);
        if (dtype == XCT_F16) return f(bp_mirror_kernel<f16_t, 96, SL>, th);
        return f(bp_mirror_kernel<bf16_t, 96, SL>, th);
    }
    if (dtype == XCT_F32) return f(bp_mirror_kernel<float, 192, SL>, th);
    if (dtype == XCT_F16) return f(bp_mirror_kernel<f16_t, 192, SL>, th);
    return f(bp_mirror_kernel<bf16_t, 192, SL>, th);
}

template <typename F>
static auto with_kernel(int path, int dtype, int win, int sl, F &&f)
{
    if (path == kPathGeneric) {
        if (dtype == XCT_F32) return f(bp_generic_kernel<float>, kBPThreads);
        if (dtype == XCT_F16) return f(bp_generic_kernel<f16_t>, kBPThreads);
        return f(bp_generic_kernel<bf16_t>, kBPThreads);
    }
    if (path == kPathMirror) return sl == 2 ? with_mirror<2>(dtype, win, f) : with_mirror<1>(dtype, win, f);
    return sl == 2 ? with_sym<2>(dtype, win, f) : with_sym<1>(dtype, win, f);
}

hipError_t launch_bp(int path, const BPBatch &b, int dtype, int sl, int grid, size_t lds, hipStream_t s)
{
    return with_kernel(path, dtype, b.win, sl,
                       [&](auto k, int threads) { return launch(k, threads, b, grid, lds, s); });
}

int bp_block_threads(int path, int sl)
{
    if (path == kPathGeneric) return kBPThreads;
    return sl == 2 ? sym_threads<2>() : sym_threads<1>();
}

int bp_max_blocks_per_cu(int path, int dtype, int win, int sl, size_t lds)
{
    return with_kernel(path, dtype, win, sl, [&](auto k, int threads) { return occupancy(k, threads, lds); });
}

}  // namespace xct
