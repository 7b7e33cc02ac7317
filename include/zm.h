/*
 * zm.h -- C ABI of libzm: Zernike moments on AMD Instinct MI355X (gfx950).
 *
 * Computes every Zernike moment Z_nm (0 <= n <= n_max, 0 <= m <= n, n - m
 * even) of eq. (1) of Al-Rawi, "Ultra-Fast Zernike Moments using FFT and GPU"
 * (arXiv 2304.14492), for batches of frames:
 *
 *   Z_nm = (n+1)/(pi eps_m) * sum_r w_r R_nm(rho_r) * (2 pi / A) * sum_a f^(rho_r, theta_a) exp(-j m theta_a)
 *
 * on an R-ring x A-angle polar grid over the frame's inscribed disk, with the
 * radial polynomials R_nm taken from the DFT relation eq. (7) (Chebyshev-U
 * samples transformed over angle, Sec. 2.1) and eps_m the optional Neumann
 * factor of eq. (14)-(15) (eps_0 = 2, else 1; 1 when normalisation is off).
 * Moments with m < 0 follow from Z_{n,-m} = conj(Z_nm) (Sec. 2) and are not
 * stored.
 *
 * Geometry (all entry points): a frame is H x W row-major; the unit disk is
 * the inscribed disk of radius D/2 pixels, D = min(H, W), centred at
 * ((W-1)/2, (H-1)/2) in pixel-centre coordinates; x points right, y up,
 * theta counter-clockwise.  The polar sample (r, a) sits at rho_r,
 * theta_a = 2 pi a / A, and takes the bilinear interpolation of the four
 * surrounding pixels; pixels outside the frame count as 0 (Sec. 2.5).
 *
 * Canonical moment order: n ascending, then m ascending over m = n mod 2,
 * n mod 2 + 2, ..., n; zm_index(n, m) gives the position.
 *
 * Conventions: every call returns a zm_status; no exception or signal
 * crosses the ABI.  Argument checks are synchronous.  Device work is
 * enqueued on the caller's HIP stream and returns before it completes;
 * a fault in it surfaces at the caller's next synchronisation (and as
 * ZM_EDEVICE from the next call that synchronises).  zm_last_error()
 * returns a thread-local description of the most recent failure.
 *
 * Diagnostics: the environment variable ZM_LOG (read once per process)
 * selects lines on stderr, "zm: <level>: <text>": 0 or unset = none,
 * 1 = every failure (the zm_last_error text), 2 = also plan and batch
 * set-up (grid sizes, resident and workspace bytes, tuned batch shape),
 * 3 = also every call that enqueues device work.
 */
#ifndef ZM_H_
#define ZM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct zm_plan_s* zm_plan_t; /* opaque; owns the resident device tables */
typedef void* zm_stream_t;           /* a hipStream_t; NULL means the null stream */

typedef enum {
    ZM_OK = 0,
    ZM_EINVAL = -1,       /* invalid argument (null pointer, bad size, bad combination) */
    ZM_ENOMEM = -2,       /* device or host allocation failed */
    ZM_EDEVICE = -3,      /* a HIP runtime call failed */
    ZM_EUNSUPPORTED = -4, /* valid request outside what the kernels support */
    ZM_EBUSY = -5         /* resource in use */
} zm_status;

/* Arithmetic of the radial projection (the dense contraction over rings).
 * The radial tables are always generated in FP64.
 *   ZM_F64    : FP64 frames, FP64 resampling / FFT / projection; FP64 moments.
 *   ZM_F32    : FP32 frames, FP32 resampling / FFT / projection; FP32 moments.
 *   ZM_BF16X2 : as ZM_F32, but the projection splits both operands into
 *               hi + lo bfloat16 parts (three products, FP32 accumulation).
 *   ZM_F16X2  : as ZM_BF16X2 with IEEE half parts (operands scaled by powers
 *               of two per table row and per frame to stay in half range). */
typedef enum { ZM_F64 = 0, ZM_F32 = 1, ZM_BF16X2 = 2, ZM_F16X2 = 3 } zm_dtype;

/* Radial quadrature of eq. (1):
 *   ZM_RING_MIDPOINT       : rho_r = (2r+1)/(2R), w_r = rho_r / R (uniform rings);
 *   ZM_RING_GAUSS_LEGENDRE : Gauss-Legendre nodes mapped to [0, 1], w_r = w_GL,r rho_r / 2. */
typedef enum { ZM_RING_MIDPOINT = 0, ZM_RING_GAUSS_LEGENDRE = 1 } zm_ring_rule;

typedef struct {
    int n_max;         /* maximum order, 0..500 (moments: 0..255)                      */
    int H, W;          /* frame rows, cols (>= 2 each; H * W * element size < 2^31 bytes) */
    zm_dtype dtype;
    int neumann;       /* nonzero: divide by eps_m (eq. (14)-(15))                     */
    int rings;         /* R; 0 selects floor(D/2)                                      */
    int angles;        /* A; 0 selects pow2ceil(max(2 n_max + 2, ceil(pi R), 32))      */
    zm_ring_rule rule;
    int device;        /* HIP device ordinal; -1 selects the current device            */
} zm_plan_desc;

typedef struct {
    int n_max, H, W, rings, angles, num_moments;
    int rings_padded;                 /* R rounded up to the projection's K step        */
    zm_dtype dtype;
    int neumann;
    zm_ring_rule rule;
    int device;
    size_t resident_bytes;            /* device memory owned by the plan                */
    size_t workspace_bytes_per_image; /* spectrum workspace one frame needs             */
    size_t workspace_bytes_fixed;     /* per-call workspace independent of batch        */
} zm_plan_info_t;

/* Number of stored moments for n_max (the pairs 0 <= m <= n <= n_max with
 * n - m even of eq. (2), Sec. 2): (n_max/2+1)(n_max/2+1) for even n_max,
 * (n_max+1)(n_max+3)/4 for odd n_max; -1 if n_max < 0. */
int zm_num_moments(int n_max);

/* Canonical position of (n, m): off(n) + m/2 with off(2p) = p(p+1),
 * off(2p+1) = (p+1)^2; -1 if n < 0, m < 0, m > n or n - m odd.  The
 * admissible pairs are those of the radial polynomials of eq. (2) (Sec. 2:
 * n >= 0, |m| <= n, n - |m| even); m < 0 is not stored (Z_{n,-m} =
 * conj(Z_nm)). */
int zm_index(int n, int m);

/* Create a plan with the default polar grid (midpoint rings, R and A as in
 * zm_plan_desc) on the current device.  Builds the FP64 radial table of
 * eq. (7) on the device, folds the quadrature weights and (n+1)/(pi eps_m)
 * into the projection operand, and keeps everything resident.  Synchronous.
 * out receives the plan (caller destroys it with zm_destroy). */
zm_status zm_plan(int n_max, int H, int W, zm_dtype dtype, int neumann, zm_plan_t* out);

/* As zm_plan with an explicit descriptor (R, A, ring rule, device).
 * Constraints: 1 <= R <= 4096; A a power of two with 32 <= A <= 4096 and
 * A >= 2 n_max + 2.  For plans with n_max > 255, or ZM_F64 plans with
 * A > 1024, the moment entry points (zm_moments, zm_spectra, zm_project,
 * zm_moments_polar, the batch calls) return ZM_EUNSUPPORTED; the table,
 * ring-node and reconstruction entry points serve them. */
zm_status zm_plan_ex(const zm_plan_desc* desc, zm_plan_t* out);

/* The plan's grid and sizes (its polar grid for eq. (1): R rings, A angles;
 * resident and workspace bytes).  ZM_EINVAL on null arguments. */
zm_status zm_plan_info(zm_plan_t plan, zm_plan_info_t* out);

/* Copy the FP64 radial table R_nm(rho_r) produced by eq. (7) (unweighted) to
 * host memory: host_out[idx * R + r], idx canonical.  n_elems must be at
 * least num_moments * R.  Synchronous. */
zm_status zm_radial_table(zm_plan_t plan, double* host_out, size_t n_elems);

/* Copy the projection operand the plan holds on the device to host memory,
 * decoded to FP64 in the layout of zm_radial_table: host_out[idx * R + r] =
 * the folded value 2(n+1)/(A eps_m) w_r R_nm(rho_r) as the projection sees it
 * (FP64, FP32, hi + lo bfloat16, or (hi + lo half) times the row's scale).
 * For checks of the precision forms against the FP64 table of eq. (7)
 * (Sec. 2.1; the stability study of Sec. 3.1).  ZM_EUNSUPPORTED for plans
 * without an operand (n_max > 255).  Synchronous. */
zm_status zm_operand_table(zm_plan_t plan, double* host_out, size_t n_elems);

/* Copy the plan's ring nodes rho_r and weights w_r (FP64, R each) to host:
 * the radial quadrature of eq. (1) on the polar grid (Sec. 2.5), midpoint
 * or Gauss-Legendre as the plan's rule says.  n_elems >= R.  Synchronous. */
zm_status zm_ring_nodes(zm_plan_t plan, double* rho_out, double* w_out, size_t n_elems);

/* Bytes of device workspace zm_moments needs for `batch` frames: the ring
 * spectra (the angular sums of eq. (1)) of every frame, plus per-frame
 * scales for ZM_F16X2.  No device call. */
zm_status zm_workspace_size(zm_plan_t plan, int batch, size_t* bytes);

/* Moments of `batch` frames by eq. (1) (Sec. 2) on the plan's polar grid:
 * the angular integral as a pruned FFT per ring of the bilinear samples
 * (Sec. 2.5), the radial one as a sum over rings against the eq. (7)
 * radial table (Sec. 2.1) with the quadrature weights and (n+1)/(pi eps_m)
 * folded in (eq. (14)-(15) when the plan has the Neumann factor).
 * Asynchronous on `stream`.
 *   d_images : device pointer, frame b at d_images + b * image_stride elements,
 *              each H x W row-major; float (FP32 dtypes) or double (ZM_F64).
 *              Only pixels within D/2 + 1.5 px of the centre are read.
 *   d_Z      : device pointer, [batch][num_moments][2] (re, im), float or double.
 *   d_ws     : device workspace of ws_bytes >= zm_workspace_size(plan, batch).
 * Overlapping calls on one plan are safe when they use distinct workspaces.
 * The plan records the completion of each call (per stream) for zm_destroy.
 * Errors: ZM_EINVAL (null pointers, batch < 0 or > 65535, image_stride <
 * H * W, workspace too small), ZM_EUNSUPPORTED (plan beyond the moment
 * kernels' limits), ZM_EDEVICE (launch failure). */
zm_status zm_moments(zm_plan_t plan, const void* d_images, int batch, long long image_stride,
                     void* d_Z, void* d_ws, size_t ws_bytes, zm_stream_t stream);

/* The two stages of zm_moments, for callers that want the ring spectra or
 * time the stages separately.  zm_spectra runs the fused resample (Sec. 2.5)
 * + angular FFT (the inner, angular sum of eq. (1), whose exp(-j m theta)
 * factor the FFT evaluates for all m at once, Sec. 2) and leaves
 * F_r[m] = sum_a f^(rho_r, theta_a) exp(-2 pi i m a / A) for
 * m = 0..n_max in the workspace (FP32, or FP64 for ZM_F64), blocked by 16
 * rings: element (frame b, ring r, m, part c: 0 = re, 1 = im) sits at
 * [b][r / 16][m][c][r % 16] over rings_padded rings; zm_project applies the
 * radial projection (the outer, radial sum of eq. (1) against the eq. (7)
 * table, Sec. 2.1) to the spectra of a preceding zm_spectra call on the
 * same workspace and stream.  zm_moments == zm_spectra followed by
 * zm_project; arguments and errors as for zm_moments. */
zm_status zm_spectra(zm_plan_t plan, const void* d_images, int batch, long long image_stride, void* d_ws,
                     size_t ws_bytes, zm_stream_t stream);
zm_status zm_project(zm_plan_t plan, int batch, void* d_Z, void* d_ws, size_t ws_bytes, zm_stream_t stream);

/* zm_moments without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): the spectra workspace is a static device array of
 * zm_static_scratch_bytes() bytes (32 MiB) that the library holds on every
 * device it runs on until the process ends.  Same arguments, layout and
 * results as zm_moments (bit-identical).  The call allocates nothing: no
 * hipMalloc / hipFree, no event creation (the completion event zm_destroy
 * checks is one made with the plan, reused when its last use has finished).
 * ZM_EINVAL if the batch needs more scratch than the array holds (the error
 * text gives the largest batch of this plan that fits: 19 frames of 4K at
 * n_max 200).  All calls on one device share the array, which keeps the
 * last call's contents: calls that overlap on one device (several streams
 * or threads) race and must be serialised by the caller. */
zm_status zm_moments_static(zm_plan_t plan, const void* d_images, int batch, long long image_stride, void* d_Z,
                            zm_stream_t stream);
size_t zm_static_scratch_bytes(void);

/* Screening of the moments of eq. (1) for non-finite values: d_counts[b]
 * receives how many of frame b's 2 * num_moments stored values (re and im)
 * are NaN or +-Inf; 0 means every moment of the frame is finite.  A NaN or
 * Inf pixel that the resampler reads (within D/2 + 1.5 px of the centre)
 * makes moments non-finite; pixels it never reads do not matter.
 *   d_Z      : device pointer, zm_moments' output for `batch` frames of this
 *              plan, [batch][num_moments][2], float or double (ZM_F64).
 *   d_counts : device pointer to int[batch], overwritten.
 * Asynchronous on `stream`; allocates nothing.  Errors: ZM_EINVAL (null
 * plan or pointers, batch < 0 or > 65535), ZM_EDEVICE (launch failure). */
zm_status zm_count_nonfinite(zm_plan_t plan, const void* d_Z, int batch, int* d_counts, zm_stream_t stream);

/* Moments from a polar image already on the grid (bypasses the resampler):
 * d_polar is [batch][R][A] (float, or double for ZM_F64). */
zm_status zm_moments_polar(zm_plan_t plan, const void* d_polar, int batch, void* d_Z, void* d_ws,
                           size_t ws_bytes, zm_stream_t stream);

/* The resampler alone (Sec. 2.5): bilinear samples of each frame on the
 * plan's polar grid, P[b][r][a] = f^(rho_r, 2 pi a / A) for r < R, a < A,
 * the inputs of the angular sum of eq. (1).  The values are the ones the
 * moment entry points sample, bit for bit, so zm_moments_polar on d_polar
 * gives the same moments as zm_moments on the frames.
 *   d_images     : device, as for zm_moments (H x W row-major frames,
 *                  frame b at d_images + b * image_stride elements; float,
 *                  or double for ZM_F64).
 *   d_polar      : device, caller-owned, [batch][R][A] of the same type,
 *                  overwritten.
 * Requires A a power of two with 256 <= A <= 4096 (ZM_EUNSUPPORTED
 * otherwise).  Asynchronous on `stream`; allocates nothing.  Errors:
 * ZM_EINVAL (null plan or pointers, batch < 0 or > 65535, image_stride <
 * H * W with batch > 1), ZM_EDEVICE (launch failure). */
zm_status zm_resample_polar(zm_plan_t plan, const void* d_images, int batch, long long image_stride, void* d_polar,
                            zm_stream_t stream);

/* ---- Batched persistent form: frames of different sizes and orders ---- */

/* One frame of a mixed batch: its plan (FP32-family dtype, n_max <= 255,
 * 512 <= angles <= 4096), the device frame (H x W float, row-major) and the
 * device output ([num_moments][2] float).  Frames sharing a plan are
 * projected together. */
typedef struct {
    zm_plan_t plan;
    const void* d_image;
    void* d_Z;
} zm_job;

typedef struct zm_batch_s* zm_batch_t; /* owns its queue, descriptors, spectra workspace and graph */

enum {
    ZM_BATCH_AUTOTUNE = 1, /* time candidate shapes once (persistent grid 1/2/4 x CUs, item order; runs
                              the batch on the given frames); the choice is cached per batch signature
                              in-process and, if the environment variable ZM_TUNE_CACHE names a file, in
                              that file */
    ZM_BATCH_NO_GRAPH = 2, /* launch directly instead of replaying a captured HIP graph */
    ZM_BATCH_PER_PLAN = 4  /* run each plan's frames as the standalone launches (resample + FFT, then
                              projection: the kernels of zm_moments) instead of the persistent kernel;
                              needs every plan's frames at one stride (e.g. slices of one array) and
                              falls back to the persistent kernel otherwise.  ZM_BATCH_AUTOTUNE also
                              times this route when the frames allow it */
};

/* Build the work queue of eq. (1) for all jobs (stage 1: fused resample +
 * ring FFT per (frame, ring tile); stage 2: radial projection per (plan
 * group, block)), allocate its device memory, optionally autotune, and
 * capture [counter reset + persistent kernel] in a HIP graph.  Synchronous.
 * Each frame's moments are bit-identical to zm_moments on that frame alone,
 * whatever the shape.  Without ZM_BATCH_AUTOTUNE the shape is grid 2 x CUs,
 * costliest tiles first (or the per-plan launches with ZM_BATCH_PER_PLAN). */
zm_status zm_batch_create(const zm_job* jobs, int njobs, int flags, zm_batch_t* out);
/* Run the batch on `stream` (asynchronous; one graph launch). */
zm_status zm_batch_run(zm_batch_t batch, zm_stream_t stream);
/* Point the batch at new frames / outputs (same plans, same order); waits for
 * the batch's last run to complete first (nothing else on the device).  A
 * batch on the per-plan route captures its launches again (their frame
 * pointers are launch arguments) and returns to the persistent kernel if the
 * new frames are not at one stride per plan. */
zm_status zm_batch_update(zm_batch_t batch, const zm_job* jobs, int njobs);
/* Wait for the batch's last run and report ZM_EDEVICE if a stage-2 item of
 * it waited past its bound (a failed dependency; never expected).  The bound
 * is 2^24 polls (each after a short sleep); the environment variable
 * ZM_BATCH_SPIN_LIMIT, read by zm_batch_create, replaces it (a small value
 * exercises this error path in tests; the kernel still finishes normally). */
zm_status zm_batch_check(zm_batch_t batch);
/* Chosen shape: persistent grid size (0 when the batch runs as per-plan
 * launches), item order (0 = costliest tiles first, 1 = natural), and the
 * queue length and device bytes owned by the batch (any pointer may be
 * NULL). */
zm_status zm_batch_config(zm_batch_t batch, int* grid, int* order, int* n_items, size_t* device_bytes);
/* Waits for the batch's last run, then frees the batch. */
zm_status zm_batch_destroy(zm_batch_t batch);
/* One-shot: create (no graph), run, synchronise, check, destroy. */
zm_status zm_moments_batch(const zm_job* jobs, int njobs, zm_stream_t stream);
/* The one-shot batch with caller-owned device memory: zm_batch_workspace_size
 * gives the bytes the jobs need (queue, descriptors, ring spectra, counters;
 * no device call), and zm_moments_batch_ws lays them out in d_ws (device,
 * 256-byte aligned, ws_bytes at least that size), uploads the queue on
 * `stream`, runs the persistent kernel there and synchronises `stream`
 * before returning.  It allocates no device memory.  Results as
 * zm_moments_batch (each frame bit-identical to zm_moments on it alone).
 * Errors: ZM_EINVAL (null or misaligned workspace, too small, bad jobs),
 * ZM_EUNSUPPORTED (a plan outside the batched form), ZM_EDEVICE. */
zm_status zm_batch_workspace_size(const zm_job* jobs, int njobs, size_t* bytes);
zm_status zm_moments_batch_ws(const zm_job* jobs, int njobs, void* d_ws, size_t ws_bytes, zm_stream_t stream);
/* The one-shot batch without any wait, for request loops that keep several
 * launches in flight: as zm_moments_batch_ws (same d_ws layout and size),
 * but the queue and descriptors go through h_stage, caller-owned pinned
 * host memory (hipHostMalloc or equivalent, 16-byte aligned) of
 * zm_batch_stage_size() bytes: the call writes them there, enqueues one
 * host-to-device copy, the persistent launch and a copy of the run's error
 * flag back into h_stage on `stream`, and returns.  d_ws and h_stage must
 * stay untouched until `stream` has passed the work; then
 * zm_batch_stage_status(h_stage) returns ZM_EDEVICE if a projection item
 * waited past its bound (ZM_OK otherwise).  Each plan records the work's
 * completion on `stream` (zm_destroy reports ZM_EBUSY until then).  It
 * allocates no device memory.  Errors: as zm_moments_batch_ws, plus
 * ZM_EINVAL for a null, misaligned or too small staging buffer. */
zm_status zm_batch_stage_size(const zm_job* jobs, int njobs, size_t* bytes);
zm_status zm_moments_batch_async(const zm_job* jobs, int njobs, void* d_ws, size_t ws_bytes, void* h_stage,
                                 size_t stage_bytes, zm_stream_t stream);
zm_status zm_batch_stage_status(const void* h_stage);

/* ---- Reconstruction (Sec. 2.2 eq. (9)), error (Sec. 2.4 eq. (13)), min-max ---- */

typedef enum { ZM_RECON_POLAR = 0, ZM_RECON_CARTESIAN = 1 } zm_recon_kind;
enum {
    ZM_RECON_ONESIDED = 1, /* sum Re(Z_nm exp(j m theta)) R_nm over stored m >= 0 once (no conj terms, no eps) */
    ZM_RECON_MINMAX = 2    /* CARTESIAN only: affine-map the result onto [min, max] of d_ref over the disk
                              (Sec. 2.3 / Sec. 3 renormalisation, per frame = per band) */
};

/* Image series of eq. (9) from moments d_Z ([batch][num_moments][2], the
 * plan's real type), FP64 accumulation, asynchronous:
 *   ZM_RECON_POLAR     : d_out [batch][R][A], f~ at the plan's polar nodes
 *                        (R_nm from the plan's eq. (7) table);
 *   ZM_RECON_CARTESIAN : d_out [batch][H][W], f~ at pixel centres with
 *                        rho <= 1, 0 outside (R_nm by the Jacobi recurrence).
 * Z_{n,-m} = conj(Z_nm) supplies the m < 0 terms; for a Neumann plan the
 * factor eps_m of eq. (14)-(15) is multiplied back, so both normalisations
 * reconstruct the same image.  d_ref (frames, [batch][H][W]) is read only
 * with ZM_RECON_MINMAX.  d_ws: zm_recon_workspace_size bytes (may be NULL
 * without ZM_RECON_MINMAX).  Output/input real type: float, double for ZM_F64. */
zm_status zm_reconstruct(zm_plan_t plan, const void* d_Z, int batch, void* d_out, int kind, int flags,
                         const void* d_ref, void* d_ws, size_t ws_bytes, zm_stream_t stream);
zm_status zm_recon_workspace_size(zm_plan_t plan, int batch, size_t* bytes);

/* Reconstruction error over the disk (pixel centres with rho <= 1) between
 * frames d_ref and reconstructions d_recon ([batch][H][W]).  host_out
 * receives batch rows of 7 doubles: eq. (13) epsilon = SSE / (f_max^2 * count),
 * eq. (10) epsilon_1 = SSE / sum f^2, SSE, f_max = max |f|, count,
 * eq. (12) epsilon_2 = sum (f - f~)^2 / f^2 over the disk pixels with f != 0
 * (the measure is singular where f = 0), and the number of disk pixels with
 * f = 0 that it leaves out.  Deterministic (fixed reduction order).
 * Synchronises the stream. */
zm_status zm_recon_error(zm_plan_t plan, const void* d_ref, const void* d_recon, int batch, double* host_out,
                         void* d_ws, size_t ws_bytes, zm_stream_t stream);

/* Embedding of Sec. 3: an N x N image is placed in a zero grid of size
 * N + floor(N (sqrt 2 - 1)) + 20 at offset floor(N (sqrt 2 - 1) / 2) + 10 in
 * both directions, so the whole image lies inside the inscribed disk.
 * zm_pad_size returns size and offset (computed exactly in integers;
 * N = 256 gives 382 and 63).  zm_embed copies a batch of n x n frames
 * (float, or double if is_double) into size x size frames. */
zm_status zm_pad_size(int n, int* size, int* offset);
zm_status zm_embed(const void* d_src, int n, int batch, void* d_dst, int is_double, zm_stream_t stream);

/* One moment Z_nm of `batch` square n_side x n_side FP32 frames (frame b at
 * d_frames + b * frame_stride elements, frame_stride >= n_side^2) by the
 * Cartesian pixel sum of eq. (6), every disk pixel centre weighted by
 * Delta^2 = (2 / n_side)^2, divided by the Neumann factor of eq. (15) when
 * `neumann` is set (eq. (14)); the constant follows eq. (1) (a constant
 * disk gives Z_00 = value * (disk pixels) Delta^2 / pi).  The 8-point
 * symmetry of the grid evaluates R_nm once per orbit of 8 pixels (Sec. 2;
 * Fig. 5 times one moment of any order this way).  0 <= n <= 500,
 * |m| <= n, n - |m| even (m < 0 returns conj(Z_n|m|), Sec. 2).  d_out
 * (device) receives batch pairs (re, im) in FP64; FP64 accumulation with a
 * fixed reduction order.  d_ws is a device workspace of at least
 * zm_cartesian_workspace_size(n_side, batch) bytes.  Runs on the calling
 * thread's current device, asynchronously on `stream`.  Errors: ZM_EINVAL
 * for bad arguments, ZM_EDEVICE for launch failures. */
zm_status zm_cartesian_workspace_size(int n_side, int batch, size_t* bytes);
zm_status zm_moment_cartesian(const void* d_frames, int n_side, int batch, long long frame_stride, int n, int m,
                              int neumann, double* d_out, void* d_ws, size_t ws_bytes, zm_stream_t stream);

/* Free a plan and its device tables.  ZM_EBUSY (nothing freed) while work
 * enqueued through the plan (zm_moments, zm_spectra, zm_project,
 * zm_moments_polar, zm_reconstruct) has not completed on its stream, or
 * while a batch object built on the plan still exists; synchronise the
 * stream / destroy the batch and call again. */
zm_status zm_destroy(zm_plan_t plan);

const char* zm_status_str(zm_status s);
const char* zm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ZM_H_ */
