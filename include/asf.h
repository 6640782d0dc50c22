/*
 * asf.h -- C ABI of the MI355X (gfx950) arbitrary-shape-surface Fresnel library.
 *
 * The library evaluates the Fourier-form Fresnel diffraction from a curved
 * source surface onto a uniform planar destination grid (Shimobaba, Masuda and
 * Ito, "Arbitrary shape surface Fresnel diffraction", Sec. 2, Eq. (7)-(9)):
 *
 *   u2(X, Y) = exp(i k (z0 + (X^2 + Y^2) / (2 z0))) / (i lambda z0)
 *            * sum_j u1_j u_I,j exp(i k [ -d_j + |x_j|^2 / (2 r0_j) - x_j . X / r0_j ])
 *
 * with k = 2 pi / lambda, r0_j = z0 - d_j, u_I,j = exp(i k d_j) (normal plane
 * wave, the default) or 1, and the destination pixel (ix, iy) at
 * X = x0 + p2x (ix - mx/2), Y = y0 + p2y (iy - my/2).  The sum is a 2D type-1
 * (non-uniform to uniform) Fourier transform of Eq. (9) with per-point
 * frequencies x_j / (lambda r0_j) (Eq. (8)); the library computes it as a
 * non-uniform FFT: an exponential-of-semicircle spreading onto a 2x oversampled
 * grid, a uniform FFT and a deconvolution (the "interpolation + uniform FFT"
 * scheme the paper relies on, Sec. 2).  The integral is a plain sum with unit
 * weights: fold any area element into u1.
 *
 * Memory: every array argument is a DEVICE pointer (hipMalloc'd or a torch
 * CUDA/HIP tensor's data pointer) unless stated otherwise.  The caller owns all
 * memory, including the workspace; the plan keeps pointers into the workspace
 * and never allocates device memory itself.  Streams are hipStream_t values
 * passed as void* (NULL = the default stream); all GPU work of a call is
 * enqueued on that stream.
 *
 * Errors: functions return ASF_OK (0) or a negative ASF_E* code; the message of
 * the calling thread's last failure is available from asf_last_error().
 * A plan is not thread-safe; distinct plans are independent.
 */
#ifndef ASF_H
#define ASF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------------- */
#define ASF_OK 0
#define ASF_EINVAL (-1)   /* null pointer, bad size, non-finite or non-positive parameter */
#define ASF_EDOMAIN (-2)  /* some r0 = z0 - d1 <= 0, or non-finite x1, y1, d1 (found on the GPU) */
#define ASF_ENOMEM (-3)   /* workspace smaller than asf_workspace_bytes() */
#define ASF_EHIP (-4)     /* a HIP runtime call failed */
#define ASF_ESIZE (-5)    /* unsupported destination grid size */
#define ASF_ENOSYS (-6)   /* operation not implemented */

/* ---- flags ----------------------------------------------------------------- */
#define ASF_FFT_FP32 0u             /* FFT stages: FP32 radix-4 x 4 on the vector ALU */
#define ASF_FFT_SPLIT_FP16 1u       /* FFT stages: DFT-16 GEMMs of FP16 hi+lo split products on MFMA, FP32 accumulation */
#define ASF_FFT_MASK 1u
/* size of the fixed device scratch array used by asf_forward_static (per GPU) */
#define ASF_STATIC_SCRATCH_BYTES ((size_t)48 << 20)
#define ASF_INCIDENT_NONE 2u        /* u_I = 1 instead of the plane wave exp(i k d1) */

typedef struct asf_plan_s *asf_plan_t;

/*
 * Optical and grid parameters.
 *   lambda    wavelength (m), > 0
 *   z0        source-to-destination distance (m), > 0 (Eq. (2)-(3))
 *   p2x, p2y  destination pitch (m), > 0
 *   mx, my    destination grid columns and rows: each a power of two in [16, 8192]
 *             (the 2x oversampled FFT length 2m must be 16^a * {1,2,4,8})
 *   tol       requested relative L2 accuracy in [1e-7, 1e-1]; sets the spreading
 *             width w = ceil(log10(1/tol)) + 2 (7 at 1e-5, so 3..9)
 *   flags     ASF_FFT_* | ASF_INCIDENT_NONE
 *   x0, y0    centre of the destination window (m), finite: pixel (ix, iy) sits at
 *             X = x0 + p2x (ix - mx/2), Y = y0 + p2y (iy - my/2); 0, 0 centres it
 *             on the axis.  An off-axis window enters the sum of Eq. (7) as an
 *             extra per-point phase -k (x1 x0 + y1 y0) / r0 and in the destination
 *             chirp; it lets several windows tile one large destination plane.
 */
typedef struct {
    double lambda, z0, p2x, p2y;
    int32_t mx, my;
    double tol;
    uint32_t flags;
    double x0, y0;
} asf_params;

/* Read-only description of a plan (sizes the kernels run at). */
typedef struct {
    int64_t n_src;        /* source points */
    int32_t mx, my;       /* destination grid */
    int32_t nfx, nfy;     /* oversampled (fine) grid, 2 mx by 2 my */
    int32_t w;            /* spreading width in fine cells */
    double beta;          /* exponential-of-semicircle shape, 2.30 w */
    int32_t tile_x, tile_y; /* spreading tile edges in fine cells */
    int32_t ntiles;       /* tiles in the fine grid */
    int64_t slot_cap;     /* capacity of the binned point list (4 n_src) */
    int32_t col_batch;    /* panel width C of the fine grid (adjacent columns stored together;
                             columns per workgroup in the first FFT pass) */
    uint32_t flags;
    /* byte offsets into the workspace of buffers tests may inspect (off_status and
     * off_cursor: the copy of the counters the latest binning used; two binnings
     * in a row use alternate copies; off_cell and off_perm are the two u32 fields of
     * 8-byte records, off_frac and off_phase the two float pairs of 16-byte records) */
    size_t off_status, off_tile_start, off_cell, off_frac, off_phase, off_perm, off_fine, off_mid;
    size_t ws_bytes;
    /* per-tile record counts (u32 [ntiles]) and slabs (u32 pairs [ntiles]: first slot,
       slot count); a tile's records are slab.first .. + min(count, slab.count) unless
       status bit 2 says the compact layout (tile_start) is in use */
    size_t off_cursor, off_slab;
    /* crowded tiles cut into slices of records (u32 [ntiles]: 0, or first partial slot
       << 8 | slices, meaningful for tiles of more records than split_meta[0]; u32 [3]:
       that threshold, the partial slots in use and the tiles no record reaches; u32
       [512]: tile << 8 | slice per slot), and the resident workgroups the cut is sized
       against (0: never cut) */
    size_t off_split, off_split_meta, off_slot_owner;
    uint32_t split_slots;
    /* per-tile flags of the last binning (u8 [ntiles], in tile order ty * ntx + tx): 1
       where some record reaches the tile, 0 where none does; then u8 [ntx], 1 for the
       tile columns holding such a tile.  When many tiles are empty the transforms
       leave those tiles' fine-grid cells as they were (the forward's column pass reads
       them as zeros), and the fine-grid columns of the tile columns flagged 0, being
       zeros, are neither transformed nor stored in the column-pass output */
    size_t off_live;
    /* 1 while the plan's transforms leave those tiles unwritten (a quarter or more of
       the tiles were empty at the last status read), else 0 */
    uint32_t skip_empty;
    /* panel width of the first FFT pass's output (element (x, ky) at ((x / P) my + ky) P + x % P):
       col_batch, or more where several first-pass workgroups fill one panel */
    int32_t mid_panel;
} asf_info;

/*
 * Bytes of device workspace a plan for n_src points with parameters *p needs.
 * Pure host computation.  Returns 0 if the arguments are invalid (see
 * asf_last_error()).
 */
size_t asf_workspace_bytes(int64_t n_src, const asf_params *p);

/*
 * Create a plan and bin the geometry (Sec. 2: the pre-phase of Eq. (8) and the
 * per-point frequencies of Eq. (9)).
 *   out        receives the plan handle (host pointer to a handle)
 *   n_src      number of source points, in [1, 2^30 - 1]
 *   x1, y1, d1 FP64 [n_src] device arrays: sample positions and surface
 *              displacement d1(x1) (m); read during the call only
 *   p          host pointer to parameters (copied)
 *   workspace  device buffer of ws_bytes >= asf_workspace_bytes(n_src, p),
 *              256-byte aligned, owned by the caller, kept alive until asf_destroy
 *   stream     hipStream_t as void*
 * Builds the FP64 host tables, uploads them, runs the geometry kernels and
 * synchronises the stream once to read the device status word.
 * Returns ASF_OK, ASF_EINVAL, ASF_ESIZE, ASF_ENOMEM, ASF_EHIP, or ASF_EDOMAIN
 * when some r0 <= 0 or a coordinate is non-finite (then *out is NULL).
 */
int asf_plan(asf_plan_t *out, int64_t n_src, const double *x1, const double *y1,
             const double *d1, const asf_params *p, void *workspace, size_t ws_bytes,
             void *stream);

/*
 * Re-bin a new geometry of the same n_src into an existing plan, asynchronously
 * (same kernels as asf_plan; no synchronisation, no host tables rebuilt).
 * Domain errors are latched in the device status word: read them with
 * asf_status().  How points are binned (one pass into per-tile slabs, or
 * counting first for crowded geometries) follows the status last read by
 * asf_plan or asf_status; the results do not depend on it, only the time.
 * Calls on one plan are ordered by the caller's stream: a later forward, adjoint
 * or asf_status sees this binning, and the binning after it reuses the counters
 * of the one before (binnings alternate between two copies), so do not issue a
 * setpts on another stream while work of the same plan is in flight.
 * Returns ASF_OK, ASF_EINVAL or ASF_EHIP.
 */
int asf_setpts(asf_plan_t plan, const double *x1, const double *y1, const double *d1,
               void *stream);

/*
 * Synchronise `stream` and read the plan's status word.  Returns ASF_OK, or
 * ASF_EDOMAIN if the last geometry had some r0 <= 0 or a non-finite coordinate
 * (those points were left out), or ASF_EHIP.
 */
int asf_status(asf_plan_t plan, void *stream);

/*
 * Forward transform, Eq. (8): u2 = A u1.
 *   u1  complex64 [n_src] device array (interleaved re, im), aligned with x1, y1, d1
 *   u2  complex64 [my][mx] device array, row-major; pixel (ix, iy) at
 *       X = x0 + p2x (ix - mx/2), Y = y0 + p2y (iy - my/2)
 * Asynchronous on `stream`; never synchronises.  u1 must be finite (the spreading
 * accumulates in fixed point; non-finite input gives an unspecified result).
 * Returns ASF_OK, ASF_EINVAL or ASF_EHIP.
 */
int asf_forward(asf_plan_t plan, const void *u1, void *u2, void *stream);

/*
 * Accumulating forward: u2 += A u1, same arguments and behaviour as asf_forward
 * except that u2 is read and added to instead of overwritten.  The fields of
 * several surfaces (one plan each, sharing the destination grid and window)
 * then sum into one destination, the superposition the paper's computer-
 * generated-hologram application needs (Sec. 4).  Calls on one u2 must be
 * ordered (the same stream, or synchronised).
 */
int asf_forward_add(asf_plan_t plan, const void *u1, void *u2, void *stream);

/*
 * For callers that cannot allocate device memory at call time (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward u2 = A u1 of asf_forward, with the same arguments, kernels and result,
 * whose fine grid and column-pass output live in the library's fixed device
 * scratch array instead of the plan's workspace.  The plan's workspace still
 * holds the binned points and tables (it is not written by this call).
 * Limit: the fine grid and the column-pass output, 8 (4 mx my + 2 mx my) bytes,
 * must fit in ASF_STATIC_SCRATCH_BYTES (48 MiB: destinations up to 1024 x 1024);
 * larger plans get ASF_ESIZE and nothing is launched.  Calls nothing that
 * allocates (no hipMalloc, hipFree or allocating library routine); the scratch
 * array exists once per GPU for the life of the process, and its address is
 * looked up on the first call on each device (the plan's device must be
 * current).  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (different streams, or different host threads) race and give wrong
 * results; order them.  The array keeps the last call's contents, which no call
 * reads before overwriting.  Asynchronous on `stream`; never synchronises.
 * Returns ASF_OK, ASF_EINVAL, ASF_ESIZE or ASF_EHIP.
 */
int asf_forward_static(asf_plan_t plan, const void *u1, void *u2, void *stream);


/*
 * Adjoint transform g1 = A^H g2 of the forward's linear map u1 -> u2: for each
 * source point j, g1_j = sum over pixels of conj(A(pixel; j)) g2(pixel), the
 * conjugate of Eq. (7)'s coefficient of u1_j (Sec. 2).  This is the backward of
 * the forward with respect to u1 (PyTorch's convention for complex gradients:
 * the gradient of u1 is A^H times the gradient of u2).  Computed as the type-2
 * (uniform to non-uniform) NUFFT: g2 times conj(Dx Dy) (the conjugate post-phase
 * over the kernel's Fourier transform), zero-padded to the fine grid, the
 * unnormalised exp(+i) DFT (rows, then columns; FP32 or split-FP16 as the plan's
 * flags say), interpolation with the same kernel at every point (no atomics),
 * times the conjugate pre-phase exp(-i phi_j).
 *   g2  complex64 [my][mx] device array, row-major (the forward's u2 layout)
 *   g1  complex64 [n_src] device array, aligned with the plan's x1, y1, d1
 * Uses the plan's workspace (do not run a forward and an adjoint of one plan
 * concurrently).  Asynchronous on `stream`; never synchronises.
 * Returns ASF_OK, ASF_EINVAL or ASF_EHIP.
 */
int asf_adjoint(asf_plan_t plan, const void *g2, void *g1, void *stream);

/* Fill *info (host pointer) with the plan's sizes.  Returns ASF_OK or ASF_EINVAL. */
int asf_plan_info(asf_plan_t plan, asf_info *info);

/*
 * Per-stage timing with HIP events recorded on the forward's stream.
 * asf_set_timing(plan, 1) makes later asf_setpts/asf_forward/asf_adjoint calls
 * record an event pair around each stage; asf_stage_times synchronises on the
 * last pair and writes up to n durations (ms, host array) in the order
 * [bin, scan, scatter, spread, fft_pass1, fft_pass2, adj_fft_pass2,
 * adj_fft_pass1, interp] (scan and scatter are the binning's fallback for
 * crowded tiles and take microseconds when it is not needed), returning how many it wrote (negative on error); a
 * stage not run since timing was enabled reads -1.  Timing adds a few
 * microseconds per stage.
 */
int asf_set_timing(asf_plan_t plan, int enable);
int asf_stage_times(asf_plan_t plan, double *ms, int n);

/* Release the plan (host memory and events; the workspace stays the caller's). */
int asf_destroy(asf_plan_t plan);

/* ---- one-dimensional profiles ---------------------------------------------- */

/*
 * The same method for a line source: sample positions x1 along one axis with
 * displacement d1(x1), onto a line of m destination pixels -- the setting of
 * the paper's profiles (Sec. 3: tilted facets, a quadratic curve).  The paper
 * gives the 1D form only by example; it is taken as Eq. (7) for a surface and
 * field that do not vary along y, with the y integral done analytically and
 * its amplitude r0 -> z0 as in the 2D amplitude approximation:
 *
 *   u2(X) = exp(i k (z0 + X^2 / (2 z0))) / sqrt(i lambda z0)
 *         * sum_j u1_j u_I,j exp(i k [ -d_j + x_j^2 / (2 r0_j) - x_j X / r0_j ])
 *
 * with X = x0 + p2 (ix - m/2).  Computed as a 1D type-1 NUFFT (same kernel,
 * width and 2x oversampling as the 2D path), one workgroup per field.
 */
typedef struct asf_line_s *asf_line_t;

/*
 * Parameters of a line plan.
 *   lambda, z0, p2  wavelength, distance, destination pitch (m), finite and > 0
 *   x0              destination window centre (m), finite
 *   m               destination pixels, a power of two in [16, 8192]
 *   tol             requested relative L2 accuracy in [1e-7, 1e-1] (w as for asf_params)
 *   flags           0 or ASF_INCIDENT_NONE
 */
typedef struct {
    double lambda, z0, p2, x0;
    int32_t m;
    double tol;
    uint32_t flags;
} asf_line_params;

/* Largest number of source points of a line plan. */
#define ASF_LINE_MAX_POINTS 16384

/*
 * Bytes of device workspace a line plan for n_src points needs (host only).
 * Returns 0 if the arguments are invalid (n_src outside [1, ASF_LINE_MAX_POINTS],
 * bad parameters; see asf_last_error()).
 */
size_t asf_line_workspace_bytes(int64_t n_src, const asf_line_params *p);

/*
 * Create a line plan: FP64 host tables (deconvolution with the 1D destination
 * phase, FFT twiddles) and one workgroup that forms each point's pre-phase and
 * frequency in FP64 (as the 2D geometry kernels do) and sorts the points by
 * their first fine cell.  Synchronises `stream` once to read the status word.
 *   out        receives the handle (host pointer)
 *   n_src      points, in [1, ASF_LINE_MAX_POINTS]
 *   x1, d1     FP64 [n_src] device arrays (m); read during the call only
 *   p          host pointer to parameters (copied)
 *   workspace  device buffer of >= asf_line_workspace_bytes(n_src, p) bytes,
 *              256-byte aligned, caller-owned, alive until asf_line_destroy
 * Returns ASF_OK, ASF_EINVAL, ASF_ESIZE, ASF_ENOMEM, ASF_EHIP, or ASF_EDOMAIN if
 * some r0 <= 0 or a coordinate is non-finite (then *out is NULL).
 */
int asf_line_plan(asf_line_t *out, int64_t n_src, const double *x1, const double *d1,
                  const asf_line_params *p, void *workspace, size_t ws_bytes, void *stream);

/*
 * Forward transform of `batch` fields through the same line geometry.
 *   u1  complex64 [batch][n_src] device array (interleaved re, im)
 *   u2  complex64 [batch][m] device array; pixel ix of field b at u2[b m + ix]
 * batch >= 1.  Asynchronous on `stream`.  The result does not depend on the
 * batch or on other fields (each field is summed in a fixed order: bitwise
 * repeatable).  Returns ASF_OK, ASF_EINVAL or ASF_EHIP.
 */
int asf_line_forward(asf_line_t plan, int32_t batch, const void *u1, void *u2, void *stream);

/* Release a line plan (host memory only). */
int asf_line_destroy(asf_line_t plan);

/* Message of the calling thread's last failure ("" if none). */
const char *asf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ASF_H */
