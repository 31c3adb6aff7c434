/*
 * xct.h - C ABI of the MI355X (gfx950) parallel-beam filtered back-projection
 * library (libxct.so).
 *
 * The operation is the per-slice reconstruction stage of the paper "Paradigm
 * Shift in Infrastructure Inspection Technology" (arXiv 2505.13955): every
 * detector row of a parallel-beam scan is reconstructed into its own slice
 * (Section V-A a, scan-row partition) by filtered back-projection, i.e. a
 * ramp-type filter along each projection row followed by back-projection of
 * the filtered rows (Section IV-B; Section V-A c, stage 2, cost
 * O(N_p N_x N_y) per slice).  Arguments follow the paper's Table I: N_p
 * projection angles, N_c detector channels, N_x x N_y slices.
 *
 * Conventions (the paper states none; these are the ones this library fixes):
 *   pixel (row i, col j) centre  x_j = (j - (N_x-1)/2) * pixel_size
 *                                y_i = (i - (N_y-1)/2) * pixel_size
 *   detector coordinate (bins)   u = (x cos th + y sin th) / det_pitch + center
 *   hat weight                   K(t) = max(0, 1 - |t|), bin n centred at u = n
 *   A[(k,n),(i,j)]               = K(u_k(x_j, y_i) - n)
 * Rows are zero outside [0, N_c): taps there contribute nothing (no clamping).
 *
 * Layouts (row-major, contiguous, no padding):
 *   sinogram  [S][N_p][N_c]   detector fastest
 *   image     [S][N_y][N_x]   column (x) fastest
 *
 * Ownership: every array pointer is a DEVICE pointer owned by the caller,
 * except xct_geometry.angles, a HOST array read during the call only.  Work is
 * enqueued on `stream` (a hipStream_t; NULL = the null stream) and the call
 * returns without synchronising; results are visible after the stream syncs.
 *
 * Device tables: the library keeps one cache of per-geometry device tables
 * (trigonometry, filter spectra, forward-projector plans, blur taps,
 * redundancy weights), built on the host in FP64.  The first call with a
 * geometry allocates its tables (hipMalloc, pinned host staging) and uploads
 * them asynchronously on that call's stream; calls on other streams wait for
 * the upload through an event.  Later calls with the same geometry allocate
 * nothing, so a call that is captured into a HIP graph must not be a
 * geometry's first.  The cache holds at most 256 entries / 1 GiB: past that
 * the least recently used entries that no call is using are freed, after a
 * device synchronisation.  xct_cache_clear() frees them all.  The library
 * allocates nothing else.
 *
 * Errors: every argument is validated before any HIP call and nothing is
 * written when a call returns an error.  Return value 0 = XCT_OK, otherwise a
 * negative xct_status.  A failed HIP launch or allocation returns XCT_EHIP;
 * faults inside kernels surface at the caller's next synchronisation.
 * All entry points are thread-safe.
 */
#ifndef XCT_H
#define XCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XCT_VERSION 10100 /* 1.1.0 */

typedef enum {
    XCT_OK = 0,
    XCT_EINVAL = -1,     /* null pointer, size <= 0, non-finite or non-positive geometry */
    XCT_EDTYPE = -2,     /* dtype or window id not supported by this entry point */
    XCT_EWORKSPACE = -3, /* workspace null, misaligned or smaller than required */
    XCT_ETOOBIG = -4,    /* a size beyond the documented limits */
    XCT_EHIP = -5        /* the HIP runtime reported an error */
} xct_status;

/* XCT_U16: raw detector counts, accepted only by xct_preprocess_filter. */
typedef enum { XCT_F32 = 0, XCT_F16 = 1, XCT_BF16 = 2, XCT_U16 = 3 } xct_dtype;

/* Filter windows W(nu) applied to the ramp |nu| on |nu| <= 1/2 (cut-off at
 * the detector Nyquist frequency).  The spatial kernels are the inverse DTFTs
 *   Ram-Lak:      h[0] = 1/4, h[even] = 0, h[odd n] = -1/(pi^2 n^2)
 *   Shepp-Logan:  h[n] = 2 / (pi^2 (1 - 4 n^2))                (W = sinc)
 *   Hann:         h[n] = h_RL[n]/2 + (h_RL[n-1] + h_RL[n+1])/4  (W = (1+cos 2 pi nu)/2) */
typedef enum { XCT_RAM_LAK = 0, XCT_SHEPP_LOGAN = 1, XCT_HANN = 2 } xct_window;

typedef void *xct_stream; /* hipStream_t */

/* One slice geometry (Table I: N_p, N_c, N_x, N_y). */
typedef struct {
    int32_t n_angles;      /* N_p >= 1                                       */
    int32_t n_det;         /* N_c >= 1                                       */
    int32_t nx, ny;        /* N_x, N_y >= 1                                  */
    double det_pitch;      /* detector bin width, > 0                        */
    double pixel_size;     /* pixel width, > 0                               */
    double center;         /* rotation axis in detector bins (finite)        */
    const double *angles;  /* HOST [n_angles] projection angles in radians  */
} xct_geometry;

/* Limits: N_c <= 8192 for the filter (FFT length 2*N_c-1 rounded up to a power
 * of two, at most 16384, held in one workgroup's LDS); N_x, N_y, N_c <= 65536,
 * N_p <= 1 << 20; S * max(N_p*N_c, N_x*N_y) < 2^62; 1/16 <= pixel_size/det_pitch <= 16;
 * |center| <= 1e6; the forward projector takes at most 65535 slices per call;
 * a back-projection launch covers fewer than 2^31 work items (64 x 64 tiles
 * times slices); xct_fbp_batch takes at most 65536 slabs.  Larger sizes
 * return XCT_ETOOBIG.  Work that needs more than 2^32 work-items in one grid
 * is split into several launches on the same stream. */

/* Windowed ramp filter of every sinogram row (Section IV-B, first step):
 *   filtered[s][k][n] = (1/det_pitch) sum_{m=0}^{N_c-1} h_W[n-m] sino[s][k][m]
 * Linear (not circular) convolution: the row is zero outside the detector.
 * Only n_angles, n_det and det_pitch of `g` are used (angles may be NULL).
 * sino: [n_slices][N_p][N_c] of sino_t; filtered: same shape, of filtered_t
 * (F16 / BF16 outputs are rounded to nearest even).  In-place
 * (filtered == sino) is allowed when both dtypes are equal. */
int xct_filter(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
               void *filtered, int32_t filtered_t, int32_t window, xct_stream stream);

/* Offset scans (Section V-A b): the sample is shifted laterally so that the
 * rotation axis sits off the detector centre, and a full turn is acquired;
 * every ray near the axis is measured twice (bin n at angle th, bin 2c - n at
 * th + pi) and the rest once.  Reconstruction weights each row by the
 * redundancy weight
 *   w[n] = 0 (t <= -1),  sin^2(pi (1 + t) / 4) (|t| < 1),  1 (t >= 1),
 *   t = (n - c) / overlap, signed positive on the detector's longer side
 * (w[n] + w[2c - n] = 1), places it on the virtual detector (the physical bins
 * and their mirror images about the axis), ramp-filters it there, and
 * back-projects the full turn through the virtual detector with weight
 * 2 pi / N_p.  For parallel beams this equals half-turn FBP on the virtual
 * detector.  Requires 2c integral, 0 <= c <= N_c - 1 and
 * 0 < overlap <= min(c, N_c - 1 - c).
 *
 * xct_offset_detector: size and axis of the virtual detector,
 *   n_virtual = 2 (N_c - 1 - c) + 1 and center_virtual = N_c - 1 - c when the
 *   longer side is right of the axis, else 2c + 1 and c.
 * xct_filter_offset: filtered [n_slices][N_p][n_virtual] of filtered_t from
 *   sino [n_slices][N_p][N_c]; n_virtual <= 8192 (else XCT_ETOOBIG); not in
 *   place.  Back-project it with the geometry's n_det = n_virtual, center =
 *   center_virtual and scale = 2 pi / N_p; angle sets of a full turn closed
 *   under quarter turns (N_p divisible by 4, uniform) take the symmetric
 *   kernel. */
int xct_offset_detector(const xct_geometry *g, int32_t *n_virtual, double *center_virtual);
int xct_filter_offset(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
                      void *filtered, int32_t filtered_t, int32_t window, double overlap,
                      xct_stream stream);

/* Pre-processing front end fused into the filter (Section V-A c, stage 2:
 * Beer-Lambert conversion, Gaussian blur, then filtering), which also regroups
 * the projection stack as acquired into one sinogram per detector row:
 *   p[s][k][n]  = -ln(max(I - D, floor) / max(F - D, floor)),
 *                 I = proj[k][row_begin + s][n], D = dark[row_begin + s][n],
 *                 F = flat[row_begin + s][n]                      (FP32: the
 *                 quotient by the hardware reciprocal of F - D, taken at
 *                 most 2^126; the logarithm by the hardware base-2
 *                 logarithm of the quotient, taken at least 2^-126, so
 *                 p <= 126 ln 2 = 87.3)
 *   b[s][k][n]  = sum_{|m| <= R} g[m] p[s][k][clamp(n + m, 0, N_c - 1)],
 *                 g[m] = exp(-m^2 / (2 sigma^2)) / sum, R = int(4 sigma + 0.5)
 *                 (sigma = 0: b = p)
 *   filtered    = xct_filter of b with the same window.
 *   proj       device [N_p][n_rows][N_c] of proj_t (XCT_U16 counts or XCT_F32)
 *   dark, flat device [n_rows][N_c] FP32 (dark current and open-beam fields)
 *   filtered   device [n_slices][N_p][N_c] of filtered_t (F32 / F16 / BF16);
 *              must not overlap proj
 * Rows row_begin .. row_begin + n_slices - 1 of the detector are processed
 * (a slab of the scan).  Errors: XCT_EINVAL for null pointers, a row range
 * outside [0, n_rows), floor below FLT_MIN (the smallest normal float),
 * sigma < 0 or non-finite; XCT_ETOOBIG for
 * R > 64 (sigma >= 16.125) or N_c > 8192; XCT_EDTYPE for other dtypes. */
int xct_preprocess_filter(const xct_geometry *g, int32_t n_rows, int32_t row_begin, int32_t n_slices,
                          const void *proj, int32_t proj_t, const float *dark, const float *flat,
                          float floor, float blur_sigma, void *filtered, int32_t filtered_t,
                          int32_t window, xct_stream stream);

/* Back-projection (Section IV-B, second step):
 *   image[s][i][j] = (accumulate ? image[s][i][j] : 0)
 *                    + scale * sum_k sum_n sino[s][k][n] K(u_k(x_j, y_i) - n)
 * Linear interpolation along the detector in FP32; FP16 / BF16 sinograms are
 * widened exactly and everything after is FP32.  Kernel choice (results agree
 * to FP32 rounding): square even slices with an angle set closed under
 * quarter turns and 2c integral take the quarter-turn symmetric kernel; any
 * other slice with 2c integral the mirror kernel (pixel pairs reflected
 * through the slice centre, u -> 2c - u); the rest the generic kernel.  FBP over a half turn uses
 * scale = pi / N_p (xct_fbp_batch applies it itself). */
int xct_backproject(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
                    float *image, float scale, int32_t accumulate, xct_stream stream);

/* Back-projection with the volume-storage epilogue of the reconstruction
 * pipeline (Section V-A c, stage 4: slices normalised by a CT-number range and
 * quantised to 16-bit unsigned integers).  Each voxel's attenuation
 *   mu = scale * (A^T sino)      (FP32, as xct_backproject computes it)
 * becomes the CT number HU = 1000 (mu - mu_water) / mu_water, and the range
 * [hu_min, hu_max] maps linearly onto the codes [0, 65535]:
 *   code = clamp(rint(fl(fl(mu * a) + b)), 0, 65535)
 * with a = fl32(1000 / mu_water * S), b = fl32((-1000 - hu_min) * S),
 * S = 65535 / (hu_max - hu_min) evaluated in FP64 in that order; fl() is one
 * FP32 rounding, rint rounds half to even, and NaN gives 0.
 *   image    device [n_slices][N_y][N_x] uint16, overwritten (half the bytes
 *            of the FP32 image)
 * Errors: XCT_EINVAL for mu_water <= 0, hu_max <= hu_min, non-finite
 * arguments or a, b that overflow FP32; otherwise as xct_backproject. */
int xct_backproject_u16(const xct_geometry *g, int32_t n_slices, const void *sino, int32_t sino_t,
                        uint16_t *image, float scale, double mu_water, double hu_min, double hu_max,
                        xct_stream stream);

/* Pixel-driven forward projector P of the least-squares problem, the exact
 * transpose of the back-projector up to its scale:
 *   P[(k,n),(i,j)] = (pixel^2 / pitch) K(u_k(x_j, y_i) - n)
 * (so that sum_n (P x)[k][n] * pitch = sum x * pixel^2 for every angle whose
 * rays all meet the detector), and
 *   sino[s][k][n] = (accumulate ? sino[s][k][n] : 0) + alpha (P image[s])[k][n]
 * with the factor pixel^2 / pitch applied here, in FP64 rounded once into
 * alpha's FP32 multiplier.  alpha = 1 gives P x; accumulating with alpha = -1
 * onto a copy of y forms the residual y - P x in one pass.  The paper uses a
 * forward model only to simulate scans for training data (Section V-B); this
 * operator is the differentiable pair's forward half.
 *   image  device [n_slices][N_y][N_x] FP32;  sino  device [n_slices][N_p][N_c] FP32
 * Three or more slices are projected four at a time from copies of the image
 * with the four slices' values side by side (and a transposed copy), made on
 * the stream in stream-ordered device memory: 32 N_x N_y bytes per group of
 * four slices, at most 1 GiB per chunk of groups (one group when a group
 * needs more), freed on the stream before the call returns; the first such
 * call on a device sets that device's default memory pool to keep up to
 * 1 GiB of freed memory between calls.
 * Deterministic (gather form, no atomics).  Errors: XCT_EINVAL for
 * non-finite alpha, XCT_ETOOBIG beyond 65535 slices or 2^31 workgroups
 * (one per group of four slices, 256 bins and up to 16 angles), XCT_EHIP
 * when the copies cannot be allocated. */
int xct_forward_project(const xct_geometry *g, int32_t n_slices, const float *image,
                        float *sino, float alpha, int32_t accumulate, xct_stream stream);

/* Residual form of xct_forward_project for the least-squares gradient:
 *   r[s][k][n] = y[s][k][n] + alpha (P image[s])[k][n]
 * (alpha = -1 gives r = y - P x), formed as one FP32 multiply-add per
 * element in the projector's store, so y is read once and needs no copy.
 *   image device [n_slices][N_y][N_x] FP32; y, r device [n_slices][N_p][N_c]
 *   FP32 (r may be y itself, updated in place).
 * Errors and memory use as xct_forward_project; XCT_EINVAL for a null y. */
int xct_forward_residual(const xct_geometry *g, int32_t n_slices, const float *image, const float *y,
                         float *r, float alpha, xct_stream stream);

/* Transpose of xct_forward_project (the back-projector scaled by
 * pixel^2 / pitch), the backward half of the differentiable pair:
 *   image[s] = (accumulate ? image[s] : 0) + alpha (P^T sino[s])
 *   sino   device [n_slices][N_p][N_c] FP32;  image  device [n_slices][N_y][N_x] FP32
 * Same kernels and arithmetic as xct_backproject with
 * scale = fl32(alpha pixel^2 / pitch).  The least-squares gradient
 * 2 P^T (P x - y) is alpha = -2 applied to the residual y - P x. */
int xct_project_adjoint(const xct_geometry *g, int32_t n_slices, const float *sino, float *image,
                        float alpha, int32_t accumulate, xct_stream stream);

/* One slab of slices sharing a geometry, for xct_fbp_batch. */
typedef struct {
    xct_geometry geom;
    int32_t n_slices;
    const void *sino; /* device [n_slices][N_p][N_c] of the batch's sino_t  */
    float *image;     /* device [n_slices][N_y][N_x] FP32, overwritten      */
    double offset_overlap; /* 0: a half-turn scan (FBP weight pi / N_p);
                              > 0: a full-turn offset scan reconstructed as
                              xct_filter_offset with this overlap, then the
                              back-projection through the virtual detector
                              with weight 2 pi / N_p                        */
} xct_slab;

/* Bytes of device workspace xct_fbp_batch needs for these slabs when the
 * filtered rows are kept as `filtered_t` (0 on invalid arguments). */
size_t xct_fbp_workspace_bytes(const xct_slab *slabs, int32_t n_slabs, int32_t filtered_t);

/* Filtered back-projection of a batch of slabs, possibly of different sizes
 * (the single-GPU analogue of the paper's grouped row partitions, Section
 * V-A b):
 *   image = (pi / N_p) A^T ((1/det_pitch) h_W * sino)      per slice
 * The filter runs over every row of every slab into `workspace` (stored as
 * filtered_t), then ONE persistent back-projection launch per kernel variant
 * (the quarter-turn symmetric kernel, the mirror kernel and the generic
 * kernel, the first two with two slices per work item or, for single-slice
 * slabs, one)
 * walks all (slab, slice, tile) work items, most expensive slab first; the
 * work counters and the table of slab descriptors also live in the
 * workspace.  Every work item is computed whole by one workgroup with the
 * variant a call with its slab alone would use, so the images equal those of
 * separate calls bit for bit.  workspace: device, 256-byte aligned,
 * at least xct_fbp_workspace_bytes(); its contents are scratch, and calls
 * that share a workspace must not overlap.  1 <= n_slabs <= 65536. */
int xct_fbp_batch(const xct_slab *slabs, int32_t n_slabs, int32_t sino_t, int32_t window,
                  int32_t filtered_t, void *workspace, size_t workspace_bytes,
                  xct_stream stream);

/* FP64 reductions of FP32 vectors for the adjoint-identity and gradient
 * checks:  *result = sum_i (double)a[i] * (double)b[i]           (xct_dot_f64)
 *          *result = sum_i ((double)a[i] - (double)b[i])^2       (xct_sqdist_f64)
 * a, b: device [n]; result: DEVICE pointer to one double.  Deterministic
 * (fixed reduction tree).  workspace: device, >= xct_reduce_workspace_bytes(). */
size_t xct_reduce_workspace_bytes(int64_t n);
int xct_dot_f64(const float *a, const float *b, int64_t n, double *result, void *workspace,
                size_t workspace_bytes, xct_stream stream);
int xct_sqdist_f64(const float *a, const float *b, int64_t n, double *result, void *workspace,
                   size_t workspace_bytes, xct_stream stream);

/* xct_dot_f64 without a workspace, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result bit for bit, with the
 * partial sums in a library-owned device array of 1024 doubles (8 KiB) on
 * each GPU it runs on, held until the process ends.  Every n >= 1 fits (a
 * reduction has at most 1024 partial sums), so no size is refused for
 * space.  Calls no hipMalloc, hipFree or allocating routine; the first call
 * on a device looks up that device's array address once.  All calls on one
 * GPU share its array: calls that overlap in time on one GPU (different
 * streams or threads with no ordering between them) race.
 *   a, b: device [n] FP32; result: DEVICE pointer to one double.
 * Errors: XCT_EINVAL for null pointers or n <= 0; XCT_EHIP if HIP fails. */
int xct_dot_f64_noalloc(const float *a, const float *b, int64_t n, double *result, xct_stream stream);

/* Static description of a status code. */
const char *xct_status_string(int status);
/* XCT_VERSION of the loaded library. */
int xct_version(void);
/* hipError_t of the most recent XCT_EHIP on the calling thread (0 if none). */
int xct_last_hip_error(void);
/* Frees the cached per-geometry device tables (call with no work in flight). */
void xct_cache_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* XCT_H */
