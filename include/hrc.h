/* hrc.h - C ABI of the MI355X (gfx950) Holographic Radiance Cascades library.
 *
 * The library computes, for a square grid of S = 2^N pixels per side, the
 * per-pixel fluence F of Eq. 1 as approximated by Holographic Radiance Cascades
 * (Section 4, Algorithm 1): per-pixel emission and attenuation in, per-pixel
 * fluence out (the problem statement of Section 3 and the image-in/grid-out
 * interface of Section 5).  Each quadrant solve builds the interval pyramid
 * T_0..T_N (traced levels 0..2, then the merge up of Section 4.1, Eq. 18-20),
 * merges the probe cascades down (Eq. 13-17, R_N = 0), and gathers R_0 at the
 * probe one pixel ahead (Algorithm 1, Lighting); the four quadrants are summed.
 * The cross blur of Eq. 21 is applied only with HRC_FLAG_BLUR.
 *
 * Conventions shared by every entry point
 *   - Grids are float32 [S][S] row-major: element (r, c) at r*S + c.
 *   - eps is the emission per unit length (the integrand of Eq. 3), sigma the
 *     attenuation coefficient sigma_t of Eq. 2.  Preconditions: finite and
 *     >= 0 (checked only with HRC_FLAG_VALIDATE).
 *   - Every tensor pointer is a DEVICE pointer on the context's device, owned
 *     by the caller and 16-byte aligned; outputs are overwritten, never
 *     accumulated.  Workspace is caller-owned device memory of at least the
 *     size reported by hrc_workspace_bytes; its contents on entry are ignored.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it; calls return without synchronising.
 *   - The forward, backward and batch-launch calls allocate nothing and free
 *     nothing.  hrc_create, hrc_set_environment (its first map) and
 *     hrc_batch_plan allocate.
 *   - Argument checks run on the host before any device call, in this order:
 *     size (HRC_ERR_SHAPE), pointers (HRC_ERR_INVALID_ARG), flags
 *     (HRC_ERR_UNSUPPORTED), workspace (HRC_ERR_WORKSPACE), context
 *     (HRC_ERR_INVALID_ARG).  A failed check
 *     enqueues nothing.  Launch failures return HRC_ERR_HIP; faults inside
 *     kernels surface at the caller's next synchronisation.
 *   - Results are deterministic: every output element has exactly one writer
 *     and no floating-point atomics are used.
 *   - A context may be used by one host thread at a time.
 */
#ifndef HRC_H
#define HRC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HRC_OK = 0,
    HRC_ERR_INVALID_ARG = -1,  /* NULL or misaligned pointer, NULL context, bad count */
    HRC_ERR_SHAPE = -2,        /* log2_size outside [HRC_MIN_LOG2, HRC_MAX_LOG2] */
    HRC_ERR_WORKSPACE = -3,    /* workspace smaller than hrc_workspace_bytes */
    HRC_ERR_HIP = -4,          /* a HIP runtime call or kernel launch failed */
    HRC_ERR_UNSUPPORTED = -5,  /* unknown flag bits, or a flag the call does not take */
    HRC_ERR_INPUT = -6,        /* HRC_FLAG_VALIDATE found a negative or non-finite input */
    HRC_ERR_TIMEOUT = -7,      /* a batch's dependency wait gave up (hrc_batch_status) */
    HRC_ERR_TOO_LARGE = -8     /* grid larger than hrc_forward_static takes */
} hrc_status;

#define HRC_MIN_LOG2 3
#define HRC_MAX_LOG2 12

/* Flags.  HRC_FLAG_VALIDATE scans eps and sigma on the device first and
 * synchronises the stream to report HRC_ERR_INPUT (debug use only).
 * HRC_FLAG_BLUR (forward and backward) applies the 1-px cross blur of Eq. 21
 * to the summed fluence: (1/8)[0 1 0; 1 4 1; 0 1 0], ignoring 4-neighbours
 * outside the grid or whose opacity 1 - exp(-sigma_t) differs from the
 * pixel's by more than 0.5, and renormalising over the weights kept; the
 * backward then starts with the blur's transpose (the kept set is piecewise
 * constant in sigma_t and adds no dLoss/d sigma_t term).
 * HRC_FLAG_QUADRANTS_{1,2,4} (forward only) choose how many quadrant solves
 * run side by side, each group reusing one set of pyramid buffers: fewer means
 * a smaller working set (it can stay in the 256 MB Infinity Cache) but more,
 * smaller launches.  Without one, all four run at once.  Results are
 * bitwise identical for every choice; the workspace size depends on it, so
 * pass the same flags to hrc_workspace_bytes. */
#define HRC_FLAG_VALIDATE 0x1u
#define HRC_FLAG_BLUR 0x2u
/* HRC_FLAG_HALF_INTERVALS (hrc_forward, hrc_backward, hrc_forward_static,
 * hrc_forward_rgb and the workspace queries): the interval pyramid is stored
 * as IEEE half floats, L and T in 16 bits each, as the paper stores it
 * (Section 5), which halves its traffic; every value is still computed in
 * FP32 and rounded to nearest once when stored.  Each stored level adds a
 * relative rounding of at most 2^-11 to what depends on it, so the fluence
 * stays within a relative N * 2^-11 of the FP32 result (about 5e-3 at
 * S = 1024) instead of 1e-4.  In hrc_backward the recomputed forward stores
 * its pyramid so while every adjoint stays FP32: every term of a gradient is a
 * term of the fluence with one factor differentiated (all of one sign for
 * emission, and for sigma_t), so each gradient element stays within
 * N * 2^-11 times the same gradient taken with abs(grad_fluence).  L above
 * 65504 (the half range) becomes infinite: the caller keeps the radiance
 * along any ray below it.  The bounce calls and the batch reject the flag. */
#define HRC_FLAG_HALF_INTERVALS 0x4u
/* HRC_FLAG_KEEP_PYRAMID (hrc_forward, and the workspace query) and
 * HRC_FLAG_REUSE_PYRAMID (hrc_backward): a reserve space between a forward
 * and its reverse.  The reverse reads the interval pyramid T_0 .. T_(N-1) of
 * the four quadrants and the cascade levels R_1 .. R_(N-1); hrc_backward
 * alone recomputes them from emission and sigma_t.  With KEEP the forward
 * computes them as the backward would and leaves them in its workspace, which
 * must then be the backward's size (hrc_workspace_bytes with KEEP returns it
 * as forward_bytes); the fluence is bitwise that of a plain forward.  With
 * REUSE the backward skips the recomputation and reads them from its
 * workspace, which must be that kept forward's workspace, for the same
 * log2_size, emission, sigma_t, environment map and HRC_FLAG_BLUR /
 * HRC_FLAG_HALF_INTERVALS bits, unwritten since by anything but backwards
 * that reuse it (a backward leaves them intact, so one kept forward serves
 * several reverses).  The gradients are then bitwise those of a plain
 * hrc_backward.  The library cannot check the pairing: a workspace that does
 * not hold a matching kept forward gives wrong gradients (every access stays
 * inside the workspace).  KEEP runs the four quadrants at once
 * (HRC_FLAG_QUADRANTS_1 or _2 with it: HRC_ERR_UNSUPPORTED).  The RGB calls
 * take the pair in the same way; the other calls reject both flags. */
#define HRC_FLAG_KEEP_PYRAMID 0x8u
#define HRC_FLAG_REUSE_PYRAMID 0x40u
#define HRC_FLAG_QUADRANTS_1 0x10u
#define HRC_FLAG_QUADRANTS_2 0x20u
#define HRC_FLAG_QUADRANTS_4 0x30u
#define HRC_FLAG_QUADRANTS_MASK 0x30u
/* hrc_batch_plan only: run a persistent kernel variant with the full register
 * budget (HRC_FLAG_BATCH_FULL) or with 64 registers (HRC_FLAG_BATCH_DENSE)
 * instead of letting the autotuner choose between them;
 * HRC_FLAG_BATCH_PERSISTENT: run every scene inside the persistent kernel
 * (none as its own kernels). */
#define HRC_FLAG_BATCH_FULL 0x100u
#define HRC_FLAG_BATCH_DENSE 0x200u
#define HRC_FLAG_BATCH_PERSISTENT 0x400u

typedef struct hrc_context hrc_context;

/* Create a context on HIP device `device`: uploads the cone-angle table of
 * Eq. 13 (A_m(jj) for m <= HRC_MAX_LOG2) to that device.  *out receives the
 * context, or NULL on failure. */
hrc_status hrc_create(int device, hrc_context **out);

/* Destroy a context (NULL-safe).  The caller must have finished all work
 * enqueued with it. */
void hrc_destroy(hrc_context *ctx);

/* Light from beyond the grid (the footnote to Section 4.2): later hrc_forward,
 * hrc_backward and hrc_profile_solve calls on this context take R_N, and every
 * angular fluence looked up outside the grid (rows outside [0, S), columns at
 * or past the far edge, the gather beyond the last column), from an
 * environment map instead of 0: the map's radiance in the direction of the
 * cone's centre v_m(jj + 1/2) times the cone's angle A_m(jj).  Outside the
 * grid is vacuum.
 *   radiance : host array of `samples` radiances at world angles 2 pi k /
 *              samples, measured from +x (increasing column) towards +y
 *              (increasing row); a direction takes the nearest sample (halfway
 *              between two: the next one counter-clockwise).  Copied.
 *   samples  : >= 1 to set the map, 0 to remove it (radiance ignored).
 * A uniform map E in vacuum gives F = 2 pi E everywhere.  The environment is a
 * constant of the backward (no gradient with respect to it).  Batches run
 * without it.  Allocates device memory on first use and copies synchronously:
 * call it when no work of this context is in flight.  Errors:
 * HRC_ERR_INVALID_ARG (NULL context, samples < 0, NULL radiance with
 * samples > 0), HRC_ERR_INPUT (a non-finite radiance), HRC_ERR_HIP. */
hrc_status hrc_set_environment(hrc_context *ctx, const float *radiance, int samples);

/* Static description of a status code (never NULL). */
const char *hrc_status_string(hrc_status s);

/* Workspace sizes in bytes for a grid of side 2^log2_size: forward needs the
 * interval pyramid of the four quadrants (Section 4.3.2: (N+3-2^-N) S^2
 * entries each) plus two cascade levels; backward additionally keeps every
 * cascade level, their adjoints and the adjoint pyramid.  Either output
 * pointer may be NULL.  Pure host function.  The forward size depends on
 * HRC_FLAG_QUADRANTS_* and HRC_FLAG_HALF_INTERVALS (with HRC_FLAG_KEEP_PYRAMID
 * it is the backward size), the backward size on HRC_FLAG_HALF_INTERVALS
 * only. */
hrc_status hrc_workspace_bytes(int log2_size, unsigned flags,
                               size_t *forward_bytes, size_t *backward_bytes);

/* Fluence of one scene (Algorithm 1, procedure Lighting, without blur).
 *   emission, sigma_t : [S][S] inputs
 *   fluence           : [S][S] output                                       */
hrc_status hrc_forward(hrc_context *ctx, int log2_size,
                       const float *emission, const float *sigma_t, float *fluence,
                       void *workspace, size_t workspace_bytes,
                       void *stream, unsigned flags);

/* hrc_forward without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same passes, launch shapes and results, bitwise,
 * as hrc_forward with the same flags, using instead a scratch array of
 * 69 MiB (72,351,744 bytes) that the library holds in every device it runs on
 * until the process ends (its address is looked up by hrc_create).  Takes
 * grids up to 2^9 per side (log2_size <= 9); larger ones return
 * HRC_ERR_TOO_LARGE before any device call.  Allocates, frees and
 * synchronises nothing; flags as hrc_forward except HRC_FLAG_VALIDATE
 * (HRC_ERR_UNSUPPORTED: it synchronises).  Every call on one device shares that
 * device's scratch, and what a call leaves there is overwritten by the next
 * (nothing in it needs clearing: every pass writes what it later reads), so
 * calls that overlap on one device race: run them on one stream, or one at a
 * time. */
hrc_status hrc_forward_static(hrc_context *ctx, int log2_size,
                              const float *emission, const float *sigma_t, float *fluence,
                              void *stream, unsigned flags);

/* Vector-Jacobian product of hrc_forward: given grad_fluence = dLoss/dF,
 * writes dLoss/d(emission) and dLoss/d(sigma_t).  The forward intervals and
 * cascades are recomputed inside the call (nothing is kept between calls; R_0,
 * which only the gather reads, is not recomputed);
 * the reverse runs the merge down from level 0 up, the merge up from level N
 * down, then the traced levels (the transposes of Eq. 7-8, 14-20 and of the
 * per-cell integral of Eq. 2-4).                                            */
hrc_status hrc_backward(hrc_context *ctx, int log2_size,
                        const float *emission, const float *sigma_t,
                        const float *grad_fluence,
                        float *grad_emission, float *grad_sigma_t,
                        void *workspace, size_t workspace_bytes,
                        void *stream, unsigned flags);

/* ---- Three radiance channels (RGB) over one medium ------------------------ */

/* The channels of a colour scene see the same medium (Section 3: channels are
 * independent; Section 5 stores radiance as a 3-vector), so one RGB solve
 * shares every transmittance between them: an interval is (L_r, L_g, L_b, T),
 * 16 bytes, where three one-channel solves move 3 x 8.  Each channel's
 * fluence equals hrc_forward on that channel's emission, bitwise.
 *   emission : [3][S][S] planes (channel c at c * S * S)
 *   sigma_t  : [S][S], shared by the channels
 *   fluence  : [3][S][S] planes, overwritten
 * Flags: HRC_FLAG_VALIDATE, HRC_FLAG_BLUR (each plane blurred as by
 * hrc_forward), HRC_FLAG_HALF_INTERVALS (the paper's own storage, Section 5:
 * the interval as four IEEE halves, 8 bytes, computed in FP32 and rounded once
 * when stored, each channel then within the relative N * 2^-11 of the FP32
 * result that hrc_forward's flag states) and HRC_FLAG_KEEP_PYRAMID (the
 * reserve space, as for hrc_forward: the workspace must then be the
 * backward's size for the same storage).  The context's environment map is
 * not applied (RGB calls run without one).
 * Workspace from hrc_workspace_bytes_rgb (pass the same flags; it takes
 * HRC_FLAG_REUSE_PYRAMID as well).  Argument checks as for hrc_forward. */
hrc_status hrc_workspace_bytes_rgb(int log2_size, unsigned flags, size_t *forward_bytes,
                                   size_t *backward_bytes);
hrc_status hrc_forward_rgb(hrc_context *ctx, int log2_size, const float *emission,
                           const float *sigma_t, float *fluence, void *workspace,
                           size_t workspace_bytes, void *stream, unsigned flags);

/* Vector-Jacobian product of hrc_forward_rgb: given grad_fluence ([3][S][S]),
 * writes grad_emission ([3][S][S]) and grad_sigma_t ([S][S]).  The reverse of
 * the RGB solve itself: its adjoint intervals are (dL_r, dL_g, dL_b, dT) and
 * its adjoint cascade levels three planes, so the medium's transmittances and
 * their adjoints are computed and moved once for the three channels.  The
 * radiance adjoints of a channel never depend on the transmittance adjoints,
 * so grad_emission's plane c equals hrc_backward's d emission for channel c
 * bitwise; grad_sigma_t gathers the channels inside the reverse (the sum of
 * three one-channel d sigma up to rounding).  Flags: HRC_FLAG_VALIDATE,
 * HRC_FLAG_BLUR, HRC_FLAG_HALF_INTERVALS (the recomputed pyramid stored as
 * halves, every adjoint FP32: each gradient element within N * 2^-11 times
 * the same gradient taken with abs(grad_fluence), as hrc_backward states),
 * HRC_FLAG_REUSE_PYRAMID (after hrc_forward_rgb with HRC_FLAG_KEEP_PYRAMID and
 * the same storage, as for hrc_backward).  Workspace: backward_bytes of
 * hrc_workspace_bytes_rgb for the same flags. */
hrc_status hrc_backward_rgb(hrc_context *ctx, int log2_size, const float *emission,
                            const float *sigma_t, const float *grad_fluence,
                            float *grad_emission, float *grad_sigma_t, void *workspace,
                            size_t workspace_bytes, void *stream, unsigned flags);

/* ---- Several diffuse bounces ----------------------------------------------- */

/* Multiple diffuse bounces (Section 4.2: the output fluence fed into another
 * iteration): bounce 0 is hrc_forward of (emission, sigma_t); bounce k > 0 uses
 * the emission eps_0 + albedo * sigma_t * F_{k-1} / (2 pi), the light that a
 * pixel scatters isotropically over the plane; the result is F of the last of
 * `bounces` (1..64) bounces.  albedo is [S][S] like the other fields (a value
 * in [0, 1) makes the bounces converge).  The context's environment, if any,
 * lights every bounce.  Flags: HRC_FLAG_VALIDATE (also checks albedo) and
 * HRC_FLAG_QUADRANTS_*; HRC_FLAG_BLUR is not supported here.  Workspace from
 * hrc_multibounce_workspace_bytes (it depends on `bounces` for the backward). */
hrc_status hrc_multibounce_workspace_bytes(int log2_size, int bounces, unsigned flags,
                                           size_t *forward_bytes, size_t *backward_bytes);
hrc_status hrc_multibounce_forward(hrc_context *ctx, int log2_size, const float *emission,
                                   const float *sigma_t, const float *albedo, int bounces,
                                   float *fluence, void *workspace, size_t workspace_bytes,
                                   void *stream, unsigned flags);

/* Vector-Jacobian product of hrc_multibounce_forward: dLoss/d(emission),
 * dLoss/d(sigma_t) (through every bounce's solve and through the sources) and
 * dLoss/d(albedo).  The bounces are recomputed inside the call and reversed
 * from the last. */
hrc_status hrc_multibounce_backward(hrc_context *ctx, int log2_size, const float *emission,
                                    const float *sigma_t, const float *albedo, int bounces,
                                    const float *grad_fluence, float *grad_emission,
                                    float *grad_sigma_t, float *grad_albedo, void *workspace,
                                    size_t workspace_bytes, void *stream, unsigned flags);

/* ---- Per-pass timing (profiling) ----------------------------------------- */

/* Pass kinds reported by hrc_profile_solve. */
typedef enum {
    HRC_PASS_SEED = 0,        /* traced levels T_0..T_2 (Section 4.2); the forward stores T_2 only */
    HRC_PASS_MERGE_UP = 1,    /* T_n from T_(n-1) (Eq. 18-20) */
    HRC_PASS_MERGE_DOWN = 2,  /* R_n from R_(n+1), T_n, T_(n+1) (Eq. 14-17), down to level 2
                                 (forward) or 1 (the reverse's recomputed forward) */
    HRC_PASS_TAIL = 3,        /* R_1 and R_0 from R_2 with their traced intervals folded on
                                 chip, the gather and the quadrant sum into F (Eq. 14-17,
                                 Algorithm 1, Lighting) */
    HRC_PASS_GATHER_ADJ = 4,  /* adjoint of the gather */
    HRC_PASS_MERGE_DOWN_ADJ = 5,
    HRC_PASS_INTERVAL_ADJ = 6,
    HRC_PASS_SEED_ADJ = 7,
    HRC_PASS_BLUR = 8,        /* cross blur (Eq. 21) */
    HRC_PASS_BLUR_ADJ = 9     /* its transpose */
} hrc_pass_kind;

/* Runs one hrc_forward (grad_fluence == NULL) or one hrc_backward (then
 * fluence is ignored) with the same kernels and launch shapes, each launched
 * with a pair of HIP events that the runtime records at that kernel's start
 * and end on `stream`; then synchronises `stream` and reports, per pass in
 * execution order, its kind, level n (-1 when not per level) and kernel
 * duration in milliseconds.  At most `max_passes` are reported; *count receives the
 * number of passes.  Argument checks as for hrc_forward / hrc_backward, plus
 * HRC_ERR_INVALID_ARG for NULL report arrays. */
hrc_status hrc_profile_solve(hrc_context *ctx, int log2_size,
                             const float *emission, const float *sigma_t, float *fluence,
                             const float *grad_fluence, float *grad_emission,
                             float *grad_sigma_t, void *workspace, size_t workspace_bytes,
                             void *stream, float *pass_ms, int *pass_kind, int *pass_level,
                             int max_passes, int *count);

/* ---- Batched forward + backward over scenes of different sizes ---------- */

/* One scene of a batch.  grad_fluence, grad_emission and grad_sigma_t may all
 * be NULL (forward only for that scene) or must all be set. */
typedef struct {
    int log2_size;
    const float *emission;
    const float *sigma_t;
    float *fluence;
    const float *grad_fluence;
    float *grad_emission;
    float *grad_sigma_t;
} hrc_scene;

typedef struct hrc_batch hrc_batch;

/* Plan a batch: copies the scene table, sizes and allocates the batch's own
 * workspace (device memory owned by the batch), and captures one batch in a
 * HIP graph.  The scenes run in one persistent kernel that works through one
 * queue of passes per XCD (accelerator complex die) of the device, each scene
 * pinned to one queue and the queues balanced by work: every block serves the
 * queue of the XCD it runs on, so a queue's passes exchange data through that
 * XCD's L2.  A queue runs its passes tile by tile in steps ordered by what each
 * pass reads and writes (a scene's independent passes share a step); the
 * scenes of a queue share a few workspace slots, the scenes of one slot
 * running one after another.  Optionally the scenes from a size up run first,
 * pass by pass, as kernels of their own in the same graph (a pass of a large
 * scene fills the GPU by itself), split over 1, 2 or 4 graph branches with a
 * workspace each whose passes overlap.  The autotuner picks that size
 * (possibly none), the queue layout (per XCD, or one queue for the whole
 * device whose steps then synchronise through an L2 write-back), the slots per
 * queue, the kernel variant, the tile sizes, the claim chunk and the branches,
 * timing each candidate batch on a stream of its own, on the caller's
 * buffers.  The scene pointers are
 * baked in: later launches read and write the same buffers; no scene's
 * outputs may overlap another scene's inputs or outputs.  flags: 0, or
 * HRC_FLAG_BATCH_FULL or HRC_FLAG_BATCH_DENSE, each optionally with
 * HRC_FLAG_BATCH_PERSISTENT (HRC_ERR_UNSUPPORTED otherwise).  Synchronises
 * `stream` first.  HRC_ERR_TIMEOUT if a dependency wait gave up while timing
 * the candidates. */
hrc_status hrc_batch_plan(hrc_context *ctx, const hrc_scene *scenes, int count,
                          unsigned flags, void *stream, hrc_batch **out);

/* Run a planned batch on `stream`: one graph launch; results are bitwise equal
 * to hrc_forward / hrc_backward on each scene (on a context without an
 * environment map: batches run without one).  Does not wait for the launch:
 * hrc_batch_status reports whether it completed every pass. */
hrc_status hrc_batch_launch(hrc_batch *batch, void *stream);

/* Synchronises `stream`, then reports HRC_ERR_TIMEOUT if, in a launch of this
 * batch since the previous hrc_batch_status call, a dependency wait of the
 * persistent kernel gave up (no progress for about a second) or a queue was
 * left unfinished: that launch's results are incomplete (every kernel still
 * ran to its end).  Clears the report.  HRC_OK otherwise; HRC_ERR_INVALID_ARG
 * for a NULL batch, HRC_ERR_HIP if a HIP call failed. */
hrc_status hrc_batch_status(hrc_batch *batch, void *stream);

/* Failure testing: with spins > 0, every dependency wait of later launches
 * waits for one group more than its step holds (a count never reached) and
 * gives up after `spins` polls, so the wait's error path runs and
 * hrc_batch_status reports HRC_ERR_TIMEOUT while every kernel still exits;
 * spins = 0 restores normal waits.  Copies synchronously: call it when no
 * launch of the batch is in flight. */
hrc_status hrc_batch_debug_waits(hrc_batch *batch, unsigned spins);

/* Bytes of device memory the batch owns (workspace, scheduler tables and state). */
size_t hrc_batch_workspace_bytes(const hrc_batch *batch);

/* What the autotuner chose for a planned batch: the persistent kernel variant
 * (0: 1024-thread blocks, four tiles side by side, full register budget; 1:
 * the same with 64 registers, twice the resident blocks; 2, 3: 256-thread
 * blocks, one tile each, full budget or 64 registers), the grid in blocks, the
 * target tile count per pass (each tile 256 threads), the tile groups a block
 * claims at once (a group is the tiles a block runs side by side), and how
 * many scenes run as kernels of their own.  Any output pointer may be NULL.
 * Pure host function; HRC_ERR_INVALID_ARG for a NULL batch. */
hrc_status hrc_batch_describe(const hrc_batch *batch, int *variant, int *grid,
                              int *target_tiles, int *chunk, int *direct_scenes);

/* The layout the autotuner chose: the persistent kernel's queues, 1 if each
 * serves one XCD (0: one queue for the whole device), the workspace slots per
 * queue (0: one per scene), and the graph branches the scenes that run as
 * kernels of their own are split over (1, 2 or 4: each branch has a workspace
 * of its own, and the branches' passes overlap, so that one branch fills the
 * GPU where another drains and ramps at a kernel boundary).  Any output
 * pointer may be NULL.  Pure host function; HRC_ERR_INVALID_ARG for a NULL
 * batch. */
hrc_status hrc_batch_queues(const hrc_batch *batch, int *queues, int *xcd_local, int *slots,
                            int *branches);

/* Every candidate the autotuner timed, in the order timed: *count receives
 * their number; for the first min(max, count), desc[8 i .. 8 i + 7] receives
 * (log2 size from which scenes ran as kernels of their own, 0 for none;
 * queues; 1 if one queue per XCD; workspace slots per queue, 0 for one per
 * scene; kernel variant; target tiles per pass; claim chunk; graph branches of
 * the direct scenes) and ms[i] the whole batch's time in milliseconds.  Pure
 * host function; HRC_ERR_INVALID_ARG for a NULL batch or count, a negative
 * max, or NULL arrays with max > 0. */
hrc_status hrc_batch_candidates(const hrc_batch *batch, int max, int *count, int *desc,
                                float *ms);

/* Destroy a batch (NULL-safe); frees its device memory and graph. */
void hrc_batch_destroy(hrc_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* HRC_H */
