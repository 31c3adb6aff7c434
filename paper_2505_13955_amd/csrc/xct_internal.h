// Internal declarations shared by the HIP sources of libxct.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/xct.h"

namespace xct {

constexpr int kInlineSlabs = 8;     // slabs a back-projection launch carries in its arguments
constexpr int kMaxSlabs = 1 << 16;  // slabs of one xct_fbp_batch call
constexpr int kTile = 64;          // back-projection tile edge (pixels)
constexpr int kBPThreads = 256;    // back-projection workgroup size
#ifndef XCT_SYM2_THREADS
#define XCT_SYM2_THREADS 512  // symmetric kernel, two slices per item: threads per workgroup
#endif
#ifndef XCT_SYM2_WAVES
#define XCT_SYM2_WAVES 4      // wavefronts per SIMD its register budget allows
#endif
constexpr int kMaxFFT = 16384;     // largest filter FFT length (LDS resident)

// Storage types of sinogram elements.
struct bf16_t { uint16_t bits; };
typedef _Float16 f16_t;

// One slab of slices as seen by the back-projection kernels.
struct BPSlab {
    const void *sino;    // [S][Np][Nc] filtered rows (dtype of the launch)
    void *image;         // [S][Ny][Nx], FP32 or (out_u16) uint16 CT-number codes
    const float2 *cs;    // [Np] (cos, sin) * pixel / pitch, FP32
    const double2 *csd;  // [Np] the same in FP64 (window anchors)
    double center;       // c, in bins
    int64_t item_begin;  // first work item of this slab
    int32_t n_angles, n_det, nx, ny;
    int32_t n_slices;
    int32_t tiles_x, tiles_y;  // tiles per slice (symmetric path: of one quadrant)
    int32_t mirror;            // 2c, an integer on the symmetric path
    float scale;
    int32_t accumulate;
    int32_t out_u16;           // store clamp(rint(fl(fl(v code_a) + code_b))) as uint16
    float code_a, code_b;
    int32_t sets;              // symmetric path: half-turn angle sets (2 for a full turn)
};

// Slabs, items and schedule of one back-projection launch.  Up to
// kInlineSlabs slab descriptors travel in the kernel arguments; a launch over
// more reads them from a device table (`table`, written on the launch's
// stream by write_slab_table before the launch).
struct BPBatch {
    BPSlab slab[kInlineSlabs];
    const BPSlab *table;    // device [n_slabs] descriptors, or nullptr (use `slab`)
    int64_t total_items;
    int64_t item_base;      // first item of a non-persistent launch (grids are split
                            // so that no launch exceeds 2^32 work-items)
    unsigned int *counter;  // persistent work counters (kXcds of them), or nullptr
    int32_t n_slabs;
    int32_t win;            // window entries per angle and window
    int32_t kb;             // angles (generic) / angle pairs (symmetric) per LDS stage
    int32_t xcd_remap;      // map consecutive items to one XCD (non-persistent launches)
};

// Accelerator complex dies of an MI355X: workgroups are dispatched to them
// round-robin, and each has its own L2.
constexpr int kXcds = 8;
// Items of a persistent launch are dealt to the XCDs in bundles of this many
// consecutive items (one 4 x 4 group of neighbouring tiles), so the
// workgroups of one XCD share detector windows in its L2.
constexpr int kXcdBundle = 16;

// Copy `n` slab descriptors (host array) into the device table `dst` with
// kernels on stream s (the descriptors travel as kernel arguments, so the
// copy is ordered on the stream and needs no host buffer to outlive the call).
hipError_t write_slab_table(BPSlab *dst, const BPSlab *src, int n, hipStream_t s);

// Back-projection kernels: any geometry; quarter-turn + mirror symmetric
// (square slices, angle sets closed under quarter turns, 2c integral); mirror
// only (any slice and angle set, 2c integral).
enum { kPathGeneric = 0, kPathSymmetric = 1, kPathMirror = 2 };

// Launch (returns hipError_t of the launch) and sizing helpers.
// `sl`: slices per work item of the symmetric kernel (1 or 2).
hipError_t launch_bp(int path, const BPBatch &b, int dtype, int sl, int grid, size_t lds, hipStream_t s);
size_t bp_generic_lds_bytes(int win, int kb);
size_t bp_sym_lds_bytes(int win, int kb, int sl);
size_t bp_mirror_lds_bytes(int win, int kb, int sl);
int bp_sym_window(int need);  // window of the symmetric kernel covering `need` (0: none)
int bp_max_blocks_per_cu(int path, int dtype, int win, int sl, size_t lds);
int bp_block_threads(int path, int sl);  // threads per workgroup of the kernel

// Front end read in the filter's load phase: raw projection stack
// [n_angles][n_rows][Nc] with dark and flat fields [n_rows][Nc].
struct PreArgs {
    const float *dark, *flat;
    const float *taps;   // [2 radius + 1] unit-sum Gaussian (radius 0: no blur)
    int32_t radius;
    int32_t n_rows, row_begin, n_angles;
    float floor;
};

struct FilterArgs {
    const void *in;    // [rows][in_len] (front end: the projection stack)
    void *out;         // [rows][Nc]
    const float *weight;  // [in_len] factors of the input samples, or nullptr
    int32_t in_first;     // output bin of input sample 0 (input zero elsewhere)
    int32_t in_len;       // input samples per row
    const float2 *tw;  // [L] exp(-2 pi i e / L)
    const float *H;    // [L] real spectrum / (L * pitch)
    int64_t rows;
    int64_t row_base;  // row of workgroup 0 (grids are split so that no launch
                       // exceeds 2^32 work-items)
    int32_t nc;
    int32_t L;
    int32_t log2L;
    PreArgs pre;
};
hipError_t launch_filter(const FilterArgs &a, int in_t, int out_t, hipStream_t s);
hipError_t launch_front_end_filter(const FilterArgs &a, int in_t, int out_t, hipStream_t s);

// Forward projector plan.  For each angle the detector coordinate is written
// as u = A v + B w + u0 (bins), with w the image axis the rays are walked along
// (rows when |cos| >= |sin|, else columns) and v the other one, so |A| >= |B|.
struct FPAngle {
    double A, B, u0;
    double invA;     // 1 / A
    float dv;        // -B / A: shift of a bin's crossing per walk step
    float hw;        // 1 / |A|: half-width of the hat along v
    float absA;
    int32_t taps;    // floor(2 hw) + 1 taps cover the hat
};
// A run of consecutive angles with the same walk axis whose strips stay close
// together, projected by one workgroup per bin block, and its staging shape
// for one ([0]) and four ([1]) slices per workgroup: walk steps staged at a
// time and LDS entries per staged step.
struct FPBlock {
    int32_t k0, count, walk, pad;
    int32_t rows[2], pitch[2];
};
constexpr int kFPAngles = 16;       // angles per block
constexpr int kFPBins = 256;        // bins per workgroup (one per thread)
constexpr int kFPLdsFloats = 8192;  // staged image floats per workgroup
// the stage's cross range is reduced over four corners per angle in one wavefront
static_assert(4 * kFPAngles <= 64, "angle block larger than one wavefront's corner reduction");

struct FPArgs {
    const float *image;  // [S][Ny][Nx]
    const float4 *quad, *quad_t;  // four slices per workgroup: [S/4][Ny][Nx] and [S/4][Nx][Ny]
    float *sino;         // [S][Np][Nc]
    const float *base;   // [S][Np][Nc] added to the scaled projection, or nullptr
    const FPAngle *ang;  // [Np]
    const FPBlock *blocks;
    int32_t n_blocks, bin_blocks;
    int32_t block_base;  // (slice group, bin block, angle block) index of the launch's first workgroup
    float scale;
    int32_t accumulate;
    int32_t n_angles, n_det, nx, ny, n_slices;
};
// Host: angle table and blocks with their staging shapes (XCT_ETOOBIG when
// some block has no one-slice shape; *four tells whether every block has a
// four-slice shape).
int fp_plan(const xct_geometry *g, std::vector<FPAngle> &ang, std::vector<FPBlock> &blocks, bool *four);
// `sl`: slices per workgroup, 1 or 4 (four read a.quad and a.quad_t, written
// by launch_forward_quads from the same image).
hipError_t launch_forward(const FPArgs &a, int sl, hipStream_t s);
hipError_t launch_forward_quads(const float *image, int n_slices, int nx, int ny, float4 *quad, float4 *quad_t,
                                hipStream_t s);

hipError_t launch_reduce(const float *a, const float *b, int64_t n, double *result,
                         double *partials, int nblocks, int sqdist, hipStream_t s);
int reduce_blocks(int64_t n);
// The allocation-free reduction's partial sums: this device's copy of the
// library's scratch array (looked up on first use), and its length.
hipError_t reduce_scratch(double **out);
int reduce_scratch_doubles();

hipError_t launch_fill_u32(unsigned int *p, int n, unsigned int v, hipStream_t s);

int device_cus();  // compute units of the current device

}  // namespace xct
