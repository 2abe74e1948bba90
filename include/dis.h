/*
 * dis.h -- Dense Inverse Search optical flow on AMD gfx950 (MI355X).
 *
 * The method is Kroeger, Timofte, Dai and Van Gool, "Fast Optical Flow using
 * Dense Inverse Search" (ECCV 2016): a coarse-to-fine loop (Alg. 1) that on
 * every scale s places a uniform grid of patches (Sec. 2.2 step 1),
 * initialises each from the coarser flow (step 2), aligns it by
 * inverse-compositional Gauss-Newton (Sec. 2.1 and Suppl. A), merges the
 * patch displacements into a dense field by the weighted average of Eq. (3)
 * (step 4) and refines that field variationally (Sec. 2.3); the finest
 * computed field is upscaled bilinearly to the input size (end of Sec. 3.1).
 *
 * Conventions used by every entry point:
 *   - Frames are grayscale intensities in [0, 1], row-major [h][pitch]
 *     (pitch in elements, pitch >= w), float32, or float64 when the handle
 *     was created with DIS_FLAG_IO_F64.
 *   - Flow is planar and dense: [2][h][w], the u (+x, columns) plane then the
 *     v (+y, rows) plane, same element type as the frames, such that
 *     I1(x + U(x)) ~= I0(x) (Eq. (1)).
 *   - Frame, flow and gradient pointers are DEVICE pointers owned by the
 *     caller.  All scratch memory is owned by the handle and allocated once,
 *     in dis_create.
 *   - Calls are asynchronous on the handle's HIP stream and do not
 *     synchronise it (except dis_debug_level, dis_autotune and dis_destroy's
 *     documented cases); the caller synchronises before reading results.
 *   - One host thread may use a handle at a time.
 *   - Internally all arithmetic is float64.
 *
 * Error codes: every int-returning call returns DIS_OK or a negative code;
 * dis_last_error() gives a readable message for the most recent failure.
 */
#ifndef DIS_H
#define DIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DIS_OK 0
#define DIS_EINVAL (-1)  /* bad parameter or NULL pointer */
#define DIS_ESIZE (-2)   /* size beyond the handle's capacity, or an image too small for a patch */
#define DIS_EHIP (-3)    /* a HIP runtime call failed; see dis_last_error */
#define DIS_ESTATE (-4)  /* call out of order (backward without a kept forward) */
#define DIS_ENOMEM (-5)  /* device allocation failed */

/* dis_params.flags */
#define DIS_FLAG_KEEP_FOR_BACKWARD 0x1u /* keep what dis_flow_backward needs */
#define DIS_FLAG_NO_GRAPH 0x2u          /* launch kernels one by one instead of replaying a HIP graph */
#define DIS_FLAG_PIXEL_CENTRE 0x4u      /* map coarse<->fine positions through pixel centres, (x+0.5)/2-0.5 */
#define DIS_FLAG_RAW_RESIDUAL 0x8u      /* Eq. (3) residual without mean normalisation */
#define DIS_FLAG_IO_F64 0x10u           /* frames, flow and gradients are float64 */
#define DIS_FLAG_STEREO 0x20u           /* rectified stereo (App. I): horizontal displacement only, v = 0 */
#define DIS_FLAG_FB_CONSISTENCY 0x40u   /* forward-backward consistent densification (App. B ii), plain calls */
#define DIS_FLAG_COLOUR 0x80u           /* RGB frames (App. B i): 3 planar channels, plain calls, patch 4..12 */

/*
 * Method parameters: Table 1 of the paper and the fixed values of Sec. 3.1.
 *   patch_size      theta_ps, >= 4 and <= 16
 *   overlap         theta_ov in [0, 1); patch stride = max(1, floor(theta_ps (1 - theta_ov)))
 *   coarsest_scale  theta_ss; -1 picks ceil(log2(2 w / (8 theta_ps))) (Sec. 3.1);
 *                   either way it is lowered until the level is >= theta_ps on both sides
 *   finest_scale    theta_sf >= 0; the flow is upscaled from this level
 *   gn_iters        theta_it >= 0, Gauss-Newton iterations per patch (fixed count)
 *   var_outer       theta_vo, fixed-point iterations of the refinement; -1 = s + 1 on scale s
 *   var_inner       theta_vi >= 1, red-black SOR sweeps per fixed-point iteration
 *   w_intensity, w_gradient, w_smooth   delta, gamma, alpha of Sec. 2.3 (5, 10, 10)
 *   sor_omega       SOR relaxation factor in (0, 2)
 *   refine          1 = run the variational refinement (Sec. 2.3), 0 = skip it
 *   flags           DIS_FLAG_* bits
 *   norm            error norm of the inverse search (App. B iii): DIS_NORM_L2
 *                   (the method of Sec. 2.1), DIS_NORM_L1 or DIS_NORM_HUBER -- in
 *                   every Gauss-Newton iteration each pixel's mean-normalised
 *                   residual e is replaced by sign(e) sqrt|e| (L1) or, for
 *                   |e| >= huber_b, by sign(e) sqrt(2 huber_b |e| - huber_b^2)
 *                   (Huber), before the least-squares step; the densification
 *                   weights of Eq. (3) keep the untransformed residual
 *   huber_b         Huber threshold on the 0..255 intensity scale (> 0)
 */
typedef struct dis_params {
    int32_t patch_size;
    double overlap;
    int32_t coarsest_scale;
    int32_t finest_scale;
    int32_t gn_iters;
    int32_t var_outer;
    int32_t var_inner;
    double w_intensity;
    double w_gradient;
    double w_smooth;
    double sor_omega;
    int32_t refine;
    uint32_t flags;
    int32_t norm;
    double huber_b;
} dis_params;

#define DIS_NORM_L2 0
#define DIS_NORM_L1 1
#define DIS_NORM_HUBER 2

typedef struct dis_handle dis_handle;

/*
 * Fill *out with a preset.  Presets 1-4 are the paper's operating points
 * (Sec. 3.3: (1) theta_sf 3, theta_it 16, theta_ps 8, theta_ov 0.3, no
 * refinement; (2) 3/12/8/0.4 with refinement; (3) 1/16/12/0.75; (4)
 * 0/256/12/0.75), all with theta_ss 5, delta 5, gamma 10, alpha 10,
 * theta_vo = s+1, theta_vi 5.  Presets 101-105 are the synthetic
 * workloads: 101 one 256x192 pair (8, 0.3, 3 levels, 8 iterations, theta_vo
 * 1); 102/103 the 1024x436 operating points (8, 0.3, 12 it) and (8, 0.5,
 * 16 it) over scales 5..3; 104 high quality (12, 0.75, scales 4..0, 128 it,
 * theta_vo 5); 105 the differentiable batch (8, 0.5, scales 3..0, 16 it,
 * theta_vo 3).  Every preset uses the L2 search (norm DIS_NORM_L2, huber_b 1).
 * Returns DIS_EINVAL for an unknown preset or NULL out.
 */
int dis_default_params(int preset, dis_params* out);

/*
 * Validate *p and create a handle for frames up to max_w x max_h and batches
 * of up to max_batch pairs, working on HIP stream `hip_stream` (a
 * hipStream_t; NULL = the default stream) of the current device.  Allocates
 * every device buffer the handle will use (the paper allocates all memory
 * once, Suppl. C).  On success *out holds the handle and DIS_OK is returned;
 * otherwise *out is NULL.  Errors: DIS_EINVAL (bad parameter, NULL p/out,
 * max sizes < patch size, max_batch < 1), DIS_ENOMEM, DIS_EHIP.
 */
int dis_create(const dis_params* p, int max_w, int max_h, int max_batch,
               void* hip_stream, dis_handle** out);

/*
 * Dense flow from I0 to I1 (Alg. 1).  I0 and I1 are w x h frames with row
 * pitch `pitch` elements; flow receives [2][h][w].  Enqueued on the handle's
 * stream.  Errors: DIS_EINVAL (NULL pointer, pitch < w, w or h < 1),
 * DIS_ESIZE (w > max_w, h > max_h, or the finest scale smaller than the
 * patch), DIS_EHIP.  With DIS_FLAG_KEEP_FOR_BACKWARD the handle keeps the
 * frames' pointers and per-scale flows for dis_flow_backward; the frames must
 * then stay unchanged until the backward call has run.  With
 * DIS_FLAG_FB_CONSISTENCY both directions run (App. B ii): each scale
 * searches I0 -> I1 and I1 -> I0, densifies each direction from its own
 * patches and the other direction's displaced patches (votes -u, residual of
 * the displaced template sampled bilinearly), refines each direction on its
 * own, and `flow` receives the I0 -> I1 flow (the other direction through
 * DIS_DBG_UREFINED_BWD).  The handle then holds two pair slots.  With
 * DIS_FLAG_COLOUR the frames are planar [3][h][pitch] (channel c at element
 * offset c * h * pitch); the search sums its normal equations over the
 * channels, Eq. (3) weighs by the norm over channels of the residuals, and
 * the refinement sums both data terms over the channels inside one robust
 * function each (App. B i).  It does not combine with
 * DIS_FLAG_FB_CONSISTENCY, batched calls or dis_flow_backward (DIS_EINVAL).
 */
int dis_compute_flow(dis_handle* h, const void* I0, const void* I1, int w, int hgt,
                     int pitch, void* flow);

/*
 * Flow for n independent pairs of possibly different sizes, one pair per
 * slot (n <= max_batch).  The arrays I0[], I1[], flow[] (device pointers)
 * and w[], hgt[], pitch[] are HOST arrays of length n.  All pairs of one
 * pyramid level are processed together: by a single persistent kernel
 * launch that takes work from a queue (launch mode bit 0 clear), or by one
 * launch per phase of the level covering every pair (bit 0 set, see
 * dis_set_tunables); the whole batch is replayed as one HIP graph per batch
 * composition.  Each pair's result is bitwise equal to
 * dis_compute_flow on that pair.  Errors as for dis_compute_flow, plus
 * DIS_ESIZE for n > max_batch.  In the persistent launch a task that waits
 * on its predecessors gives up after a bounded wait (about a second, which
 * a working queue never reaches); the call then writes NaN into every flow
 * of the batch, and DIS_DBG_WAIT_ERRORS counts the launches concerned.
 */
int dis_compute_flow_batched(dis_handle* h, int n, const void* const* I0,
                             const void* const* I1, const int* w, const int* hgt,
                             const int* pitch, void* const* flow);

/*
 * Gradient of a scalar loss with respect to both frames, given
 * grad_flow = dL/dflow ([2][h][w], device) for the most recent
 * dis_compute_flow on this handle (which must have run with
 * DIS_FLAG_KEEP_FOR_BACKWARD).  Writes dL/dI0 and dL/dI1 ([h][w], dense,
 * pitch = w) into caller buffers.  Each scale coarser than the finest is
 * recomputed from its kept patch records before its adjoint runs; the
 * finest scale's SOR states, weight sums, warped frame and linearisation are
 * the ones the forward wrote into the same one-scale buffers as it ran.
 * Scratch stays bounded by one scale.  Errors: DIS_EINVAL (NULL pointer, or
 * more Gauss-Newton iterations than the reverse search keeps in 64 KB of
 * LDS: 134 for 8x8 patches, 142 for 12x12, 74 for 16x16; the message gives
 * the limit), DIS_ESTATE (no kept forward), DIS_EHIP.
 */
int dis_flow_backward(dis_handle* h, const void* grad_flow, void* grad_I0, void* grad_I1);

/*
 * Time the result-invariant launch choices (lanes per patch in the search,
 * tile shape of the refinement, launch modes) on replays of the most recent
 * forward call on h, keep the fastest, and append them to the JSON file
 * `cache_path` (NULL = no file).  The replays read that call's frames again
 * -- they must still be allocated and unchanged -- and write their flow into
 * temporary buffers of their own (the caller's flow buffers are not
 * touched).  Synchronises the stream.  Errors: DIS_ESTATE (no forward call
 * yet), DIS_ENOMEM, DIS_EHIP.
 */
int dis_autotune(dis_handle* h, const char* cache_path);

/*
 * Set the launch choices that do not change results (for tests and the
 * autotuner): lanes_per_patch[s] (HOST array of 16, or NULL = automatic for
 * every scale) is the number of lanes sharing one patch in the search on
 * scale s (0 = automatic, else 4, 8, 16, 32 or 64 where compiled for the patch
 * size);
 * refine_tile picks the refinement tile (core width x height, threads) of the
 * per-phase launches: 0: 32x16/256, 1: 16x16/256, 2: 64x8/256,
 * 3: 16x16/1024, 4: 32x16/1024, 5: 16x16/512, 6: 32x16/512, 7: 8x8/512,
 * 8: 16x8/512, 9: 8x8/256, 10: 8x4/384, and with no LDS copy of U (two blocks
 * per compute unit) 11: 32x16/512, 12: 16x16/512.  launch_mode bit 0: 0 runs each scale as one
 * persistent launch over a task queue (refining with tile 0, or with tile 1
 * when that is the chosen tile and the search is the grey L2 one), 1 as one
 * launch per phase; bit 1 set
 * turns on the single-workgroup path: a scale of at most 256 horizontal
 * pixel pairs (1024 with bit 4 also set) is densified and refined, every
 * fixed-point step, by one block instead of tiles; bit 2 set makes dis_flow_backward reverse the SOR
 * sweeps with one launch per half sweep (a plain reference form) instead of
 * one tiled launch per fixed-point step; bit 3 set makes every forward
 * refinement launch recompute the linearisation from the level images
 * instead of the scale's first launch storing it for the later ones (less
 * HBM traffic, more arithmetic per launch); bit 5 exists to test the
 * failure path of the persistent launch: every wait there that would block
 * gives up at once, as a timed-out wait does (the flow becomes NaN); bit 6
 * set runs the per-phase refinement of a scale whose tiles number at least
 * twice the compute units with the lean tile of the same core and threads
 * (tile 6 -> 11, 5 -> 12) where there is one.  Every
 * other choice gives
 * bitwise-identical flow (gradients agree to rounding: they are summed with
 * atomics).  Synchronises the stream and drops cached launch
 * plans.  Errors: DIS_EINVAL.
 */
int dis_set_tunables(dis_handle* h, const int* lanes_per_patch, int refine_tile, int launch_mode);

/*
 * Read back the launch choices in force (after dis_autotune, say): any of
 * the HOST pointers may be NULL; lanes_per_patch receives 16 ints.
 * Errors: DIS_EINVAL (h NULL).
 */
int dis_get_tunables(const dis_handle* h, int* lanes_per_patch, int* refine_tile, int* launch_mode);

/* Message for the most recent failing call on h (or on a NULL handle). */
const char* dis_last_error(const dis_handle* h);

/* Move the handle to another HIP stream.  Errors: DIS_EINVAL. */
int dis_set_stream(dis_handle* h, void* hip_stream);

/*
 * Copy an intermediate of the most recent forward call on slot 0 at scale s
 * into the HOST buffer dst of `bytes` bytes (float64 values).  Synchronises
 * the stream.  `what`: DIS_DBG_J0/J1 the level images [H_s][W_s] (0..255
 * scale), DIS_DBG_UINIT [N][2] patch initialisations, DIS_DBG_UPATCH [N][2]
 * patch displacements after the reset test, DIS_DBG_UDENSE [2][H_s][W_s]
 * densified flow, DIS_DBG_UREFINED [2][H_s][W_s] flow after refinement,
 * DIS_DBG_INFO int32 {W_s, H_s, N, nx, ny, stride} (24 bytes),
 * after dis_flow_backward: DIS_DBG_GRAD_J0/J1 [H_s][W_s] dL/d(level image),
 * DIS_DBG_GRAD_U [2][H_s][W_s] dL/d(refined flow of scale s),
 * DIS_DBG_GRAD_PATCH [N][4] dL/d(patch u, v, mean residual, unused),
 * DIS_DBG_UREFINED_BWD [2][H_s][W_s] the backward (frame 1 -> 0) flow of a
 * forward-backward consistent call,
 * DIS_DBG_WAIT_ERRORS int32: how many persistent launches of that call gave
 * up waiting on their task queue (0 unless something is broken).
 * Errors: DIS_EINVAL (bad what/s or NULL), DIS_ESIZE (bytes too small),
 * DIS_ESTATE (scale not computed), DIS_EHIP.
 */
#define DIS_DBG_J0 0
#define DIS_DBG_J1 1
#define DIS_DBG_UINIT 2
#define DIS_DBG_UPATCH 3
#define DIS_DBG_UDENSE 4
#define DIS_DBG_UREFINED 5
#define DIS_DBG_INFO 6
#define DIS_DBG_WAIT_ERRORS 7
#define DIS_DBG_GRAD_J0 8
#define DIS_DBG_GRAD_J1 9
#define DIS_DBG_GRAD_U 10
#define DIS_DBG_GRAD_PATCH 11
#define DIS_DBG_UREFINED_BWD 12   /* with DIS_FLAG_FB_CONSISTENCY: the backward direction's refined flow */
int dis_debug_level(dis_handle* h, int s, int what, void* dst, size_t bytes);

/*
 * Per-kernel timing.  dis_profile_enable(h, 1) makes the following forward
 * calls launch their kernels one by one with a HIP event recorded on the
 * handle's stream before and after each launch; dis_profile_enable(h, 0)
 * returns to graph replay.  dis_profile_read synchronises the stream, folds
 * the recorded events into per-kernel totals, writes up to `max` entries into
 * out[] (host array), sets *n to the number of kernels seen and clears the
 * totals.  `bytes` and `flops` are the algorithmic (compulsory) memory traffic
 * and floating-point work of all launches of that kernel, from the sizes of
 * the arrays each launch must read and write and the operation counts of its
 * arithmetic (see the per-kernel models in the host source).
 * Errors: DIS_EINVAL (NULL), DIS_EHIP.
 */
typedef struct dis_kernel_stat {
    char name[32];
    int32_t launches;
    double total_ms;
    double bytes;
    double flops;
} dis_kernel_stat;
int dis_profile_enable(dis_handle* h, int on);
int dis_profile_read(dis_handle* h, dis_kernel_stat* out, int max, int* n);

/* Release the handle and its device memory (allocated once in dis_create,
 * as Suppl. C describes); NULL is ignored.  Synchronises the handle's stream
 * first, so pending work finishes before memory goes. */
void dis_destroy(dis_handle* h);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the flow
 * of dis_compute_flow without a handle.  Every intermediate buffer lives in
 * one static device array of DIS_NOALLOC_SCRATCH_BYTES bytes that each GPU
 * the library runs on holds until the process ends; this call never calls
 * hipMalloc or hipFree.  p, I0, I1, w, hgt, pitch and flow are as for
 * dis_create and dis_compute_flow (device frames and flow, caller-owned);
 * the kernels are enqueued one by one (no graph) on `hip_stream` of the
 * current device, without synchronising it.  The flow is bitwise equal to
 * dis_compute_flow's for the same parameters and frames.
 * All calls on one GPU share its array, which keeps the last call's
 * contents: calls that overlap on one GPU (concurrent streams, or host
 * threads) race and give wrong flow.  Calls from several host threads are
 * serialised on the host, not on the GPU.
 * Errors: DIS_EINVAL (bad parameter, NULL pointer, pitch < w, or a flag
 * this call does not take: DIS_FLAG_KEEP_FOR_BACKWARD,
 * DIS_FLAG_FB_CONSISTENCY, DIS_FLAG_COLOUR), DIS_ESIZE (the frame's
 * buffers need more than DIS_NOALLOC_SCRATCH_BYTES -- about 104 bytes per
 * pixel of the finest processed scale plus its coarser scales, e.g. fine
 * for 1024x436 at theta_sf 0 -- or the finest scale is smaller than the
 * patch), DIS_EHIP.  Messages through dis_last_error(NULL).
 */
#define DIS_NOALLOC_SCRATCH_BYTES (64u << 20)
int dis_compute_flow_noalloc(const dis_params* p, const void* I0, const void* I1, int w, int hgt,
                             int pitch, void* flow, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* DIS_H */
